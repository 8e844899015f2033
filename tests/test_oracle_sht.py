"""Pins of the oracle's spherical harmonic transforms against mathematics.

Nothing here compares the oracle with itself: every expected value comes from
a closed form, a library routine (numpy Legendre series, numpy Gauss-Legendre
nodes, scipy spherical harmonics), a textbook series evaluated in 60-digit
arithmetic, or an exact identity (adjointness, equal-area ring placement).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy.special import sph_harm_y

import dmwf_inputs as inp
import oracle

PI = math.pi


# --------------------------------------------------------------------------
# HEALPix ring geometry
# --------------------------------------------------------------------------
def test_nside1_pixel_centres():
    """Nside = 1: the twelve base pixels (Gorski et al. 2005, Fig. 3 / Table 1)."""
    th, ph = oracle.pixel_angles(1)
    z = np.cos(th)
    np.testing.assert_allclose(z[:4], 2.0 / 3.0, atol=1e-15)
    np.testing.assert_allclose(z[4:8], 0.0, atol=1e-15)
    np.testing.assert_allclose(z[8:], -2.0 / 3.0, atol=1e-15)
    np.testing.assert_allclose(ph[:4], PI / 4 + np.arange(4) * PI / 2, atol=1e-15)
    np.testing.assert_allclose(ph[4:8], np.arange(4) * PI / 2, atol=1e-15)
    np.testing.assert_allclose(ph[8:], PI / 4 + np.arange(4) * PI / 2, atol=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 64])
def test_ring_layout_equal_area(nside):
    """Rings tile RING order and every ring centre splits the cap above it in equal-area pixels.

    The spherical cap above z has area 2 pi (1 - z); for a HEALPix ring centre
    it holds the pixels of all rings above plus half of this ring.
    """
    z, st, nph, p0, start = oracle.rings(nside)
    npix = 12 * nside * nside
    assert nph.sum() == npix
    np.testing.assert_array_equal(start[1:], np.cumsum(nph)[:-1])
    assert start[0] == 0
    omega = 4 * PI / npix
    half = 2 * nside  # rings 1..2N are the north half and the equator
    lhs = 2 * PI * (1 - z[:half])
    rhs = omega * (start[:half] + nph[:half] / 2.0)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-15)
    # mirror symmetry
    np.testing.assert_allclose(z, -z[::-1], atol=1e-15)
    np.testing.assert_array_equal(nph, nph[::-1])
    np.testing.assert_allclose(st * st + z * z, 1.0, rtol=1e-15)
    # pixels of a ring are evenly spaced around the full circle
    th, ph = oracle.pixel_angles(nside)
    for k in [0, nside - 1, 2 * nside - 1, 4 * nside - 2]:
        seg = ph[start[k]:start[k] + nph[k]]
        np.testing.assert_allclose(np.diff(seg), 2 * PI / nph[k], rtol=1e-13)


def test_ring_layout_matches_input_generator():
    """The oracle's ring table and the workload generator's agree (two independent codes)."""
    for nside in (4, 32):
        z, st, nph, p0, start = oracle.rings(nside)
        z2, nph2, p02, start2 = inp.ring_layout(nside)
        np.testing.assert_allclose(z, z2, atol=1e-15)
        np.testing.assert_array_equal(nph, nph2)
        np.testing.assert_allclose(p0, p02, atol=1e-15)
        np.testing.assert_array_equal(start, start2)


# --------------------------------------------------------------------------
# Normalised associated Legendre functions lambda_lm
# --------------------------------------------------------------------------
def _closed_forms(x):
    s = math.sqrt(1 - x * x)
    return {
        (0, 0): 1 / math.sqrt(4 * PI),
        (1, 0): math.sqrt(3 / (4 * PI)) * x,
        (1, 1): -math.sqrt(3 / (8 * PI)) * s,
        (2, 0): math.sqrt(5 / (16 * PI)) * (3 * x * x - 1),
        (2, 1): -math.sqrt(15 / (8 * PI)) * s * x,
        (2, 2): 0.25 * math.sqrt(15 / (2 * PI)) * s * s,
        (3, 0): math.sqrt(7 / (16 * PI)) * (5 * x ** 3 - 3 * x),
        (3, 1): -(1 / 8) * math.sqrt(21 / PI) * s * (5 * x * x - 1),
        (3, 2): 0.25 * math.sqrt(105 / (2 * PI)) * s * s * x,
        (3, 3): -(1 / 8) * math.sqrt(35 / PI) * s ** 3,
    }


@pytest.mark.parametrize("x", [1.0, 0.97, 0.5, 0.1, 0.0, -0.3, -0.999])
def test_lambda_closed_forms(x):
    """Textbook Y_lm(theta, 0) for l <= 3, Condon-Shortley phase."""
    st = math.sqrt((1 - x) * (1 + x))
    ref = _closed_forms(x)
    for m in range(4):
        lam = oracle.lambda_lm(m, x, st, 3)
        for l in range(m, 4):
            assert lam[l - m] == pytest.approx(ref[(l, m)], abs=1e-15, rel=1e-14)


def test_lambda_zonal_vs_legendre_series():
    """lambda_l0 = sqrt((2l+1)/4pi) P_l(x), P_l from numpy's Legendre series."""
    lmax = 300
    for x in [0.9999, 0.7, 0.123, -0.45, -0.99]:
        st = math.sqrt((1 - x) * (1 + x))
        lam = oracle.lambda_lm(0, x, st, lmax)
        for l in (0, 1, 7, 64, 150, 300):
            c = np.zeros(l + 1)
            c[l] = 1.0
            ref = math.sqrt((2 * l + 1) / (4 * PI)) * npleg.legval(x, c)
            assert lam[l] == pytest.approx(ref, abs=1e-13, rel=1e-11)


def test_lambda_orthonormal_gauss_legendre():
    """2 pi int lambda_lm lambda_l'm dx = delta_ll' on Gauss-Legendre nodes (exact for degree < 2n)."""
    lmax = 40
    xs, ws = npleg.leggauss(lmax + 2)
    for m in range(lmax + 1):
        L = np.array([oracle.lambda_lm(m, x, math.sqrt(1 - x * x), lmax) for x in xs])
        G = 2 * PI * (L.T * ws) @ L
        np.testing.assert_allclose(G, np.eye(lmax - m + 1), atol=1e-13)


def test_lambda_sectoral_log_magnitude_polar():
    """|lambda_ll| = sqrt((2l+1)!/(4 pi)) / (2^l l!) sin^l theta, compared in log2 at polar rings of Nside 1024.

    Values are far below the FP64 range (down to ~2^-42000); the oracle carries them as mantissa * 2^e.
    """
    for r in (1, 2, 17, 700):
        z, st, *_ = oracle.ring(1024, r)
        for l in (1, 10, 300, 2048, 4095):
            mt, ex = oracle.lambda_lm_scaled(l, z, st, l)
            got = math.log2(abs(mt[0])) + int(ex[0])
            ref = (0.5 * math.log((2 * l + 1) / (4 * PI)) + 0.5 * math.lgamma(2 * l + 1)
                   - l * math.log(2) - math.lgamma(l + 1) + l * math.log(st)) / math.log(2)
            assert got == pytest.approx(ref, abs=1e-9 * max(1.0, abs(ref)))
            assert np.sign(mt[0]) == (-1) ** l


def _lambda_series(l, m, onemz):
    """lambda_lm from P_l^m(x) = (-1)^m (l+m)!/((l-m)! 2^m m!) (1-x^2)^{m/2} 2F1(m-l, m+l+1; m+1; (1-x)/2).

    The hypergeometric series terminates; summed in 60-digit arithmetic.
    Returns (sign, log2 |lambda_lm|).
    """
    mp.mp.dps = 60
    u = mp.mpf(onemz)
    zz = u / 2
    s, term = mp.mpf(0), mp.mpf(1)
    for k in range(0, l - m + 1):
        s += term
        term *= mp.mpf((m - l + k) * (m + l + 1 + k)) / ((m + 1 + k) * (k + 1)) * zz
        if term == 0 or abs(term) < mp.mpf(10) ** -55 * abs(s):
            break
    sin2 = u * (2 - u)
    logabs = (0.5 * mp.log((2 * l + 1) / (4 * mp.pi)) + 0.5 * (mp.loggamma(l + m + 1) - mp.loggamma(l - m + 1))
              - m * mp.log(2) - mp.loggamma(m + 1) + m / 2 * mp.log(sin2) + mp.log(abs(s)))
    sign = (-1) ** m * (1 if s > 0 else -1)
    return sign, float(logabs / mp.log(2))


@pytest.mark.parametrize("nside,r,pairs", [
    (1024, 3, [(2048, 1), (2048, 10), (2048, 30), (500, 200), (2048, 300), (1500, 700)]),
    (1024, 40, [(2048, 60), (2048, 90), (1000, 400)]),
    (256, 2, [(512, 5), (512, 100)]),
])
def test_lambda_polar_vs_hypergeometric_series(nside, r, pairs):
    """Non-sectoral polar values, including ones far below the FP64 range."""
    z, st, *_ = oracle.ring(nside, r)
    onemz = r * r / (3.0 * nside * nside)
    for l, m in pairs:
        sign, ref = _lambda_series(l, m, onemz)
        mt, ex = oracle.lambda_lm_scaled(m, z, st, l)
        got = math.log2(abs(mt[-1])) + int(ex[-1])
        assert np.sign(mt[-1]) == sign
        assert got == pytest.approx(ref, abs=3e-11 * max(1.0, abs(ref)) + 1e-10)


# --------------------------------------------------------------------------
# Synthesis and adjoint
# --------------------------------------------------------------------------
def _brute_synth(alm, nside, lmax):
    th, ph = oracle.pixel_angles(nside)
    out = np.zeros(th.size)
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            k = oracle.alm_index(l, m, lmax)
            Y = sph_harm_y(l, m, th, ph)
            if m == 0:
                out += alm[k, 0] * Y.real
            else:
                out += 2.0 * ((alm[k, 0] + 1j * alm[k, 1]) * Y).real
    return out


def _brute_adjoint(mp_, nside, lmax):
    th, ph = oracle.pixel_angles(nside)
    out = np.zeros((oracle.n_alm(lmax), 2))
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            k = oracle.alm_index(l, m, lmax)
            v = np.sum(mp_ * np.conj(sph_harm_y(l, m, th, ph)))
            out[k] = v.real, v.imag
    return out


@pytest.mark.parametrize("nside,lmax", [(1, 2), (2, 5), (4, 11), (8, 16), (8, 23)])
def test_synthesis_vs_scipy_direct_sum(nside, lmax):
    """Direct sum of a_lm Y_lm with scipy's Y_lm at every pixel centre (lmax up to 3N-1: polar aliasing)."""
    a = inp.random_alm(lmax, 10 + nside)
    a[:lmax + 1, 1] = 0.0
    got = oracle.alm2map(a, nside, lmax)
    ref = _brute_synth(a, nside, lmax)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("nside,lmax", [(2, 5), (4, 11), (8, 20)])
def test_adjoint_vs_scipy_direct_sum(nside, lmax):
    r = inp.random_map(nside, 3 + nside)
    got = oracle.adjoint(r, nside, lmax)
    ref = _brute_adjoint(r, nside, lmax)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("nside,lmax", [(16, 32), (16, 47), (32, 64)])
def test_adjointness(nside, lmax):
    """<Y a, r>_pix = <a, Y^H r>_alm with m > 0 counted twice."""
    a = inp.random_alm(lmax, 5)
    a[:lmax + 1, 1] = 0.0
    r = inp.random_map(nside, 6)
    lhs = float(np.dot(oracle.alm2map(a, nside, lmax), r))
    rhs = oracle.alm_dot(a, oracle.adjoint(r, nside, lmax), lmax)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_quadrature_near_inverse():
    """Omega Y^H Y is close to the identity for band-limited fields (HEALPix quadrature, lmax <= 2N)."""
    nside, lmax = 16, 24
    a = inp.random_alm(lmax, 9)
    a[:lmax + 1, 1] = 0.0
    back = (4 * PI / (12 * nside * nside)) * oracle.adjoint(oracle.alm2map(a, nside, lmax), nside, lmax)
    assert np.linalg.norm(back - a) < 0.02 * np.linalg.norm(a)


def test_sampled_entry_points_match_full():
    nside, lmax = 8, 16
    a = inp.random_alm(lmax, 11)
    a[:lmax + 1, 1] = 0.0
    full = oracle.alm2map(a, nside, lmax)
    rl = [1, 5, 16, 30]
    part = oracle.alm2map_rings(a, nside, lmax, rl)
    z, st, nph, p0, start = oracle.rings(nside)
    ref = np.concatenate([full[start[r - 1]:start[r - 1] + nph[r - 1]] for r in rl])
    np.testing.assert_array_equal(part, ref)
    mp_ = inp.random_map(nside, 12)
    fa = oracle.adjoint(mp_, nside, lmax)
    sub = oracle.adjoint_m(mp_, nside, lmax, [0, 3, 16])
    for m, v in sub.items():
        k0 = oracle.alm_index(m, m, lmax)
        np.testing.assert_array_equal(v, fa[k0:k0 + lmax - m + 1])
