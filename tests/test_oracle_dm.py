"""Pins of the oracle's dual messenger (paper Algorithm 2) against the Wiener filter equation.

The iteration is checked against dense linear algebra (the plain definition
of its fixed points), against an exact-transform 1-D toy where the paper's
flat-sky algebra holds verbatim, and against properties the paper states
(unconditional contraction within a level, the effect of beta, chi^2
minimality).  Planted mistakes in the oracle show that the pins catch the
plausible slips (N instead of N_bar in the pixel step, a missing sigma in the
harmonic step, the literal non-residual harmonic step on HEALPix).
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import dmwf_inputs as inp
import oracle
from oracle import dense, dm


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def sphere_problem(name="cfg1", nside=8, lmax=None, index=0):
    p = inp.make_problem(name, nside=nside, lmax=lmax, index=index)
    T = oracle.SphereTransforms(nside, p.lmax)
    d = p.data_map(T.synth(p.alm_true))
    return p, T, d, p.ninv


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


class Toy1D:
    """Periodic 1-D grid of odd length n with exact Fourier transforms (Omega Y^H Y = 1)."""

    def __init__(self, n):
        assert n % 2 == 1
        self.n = self.npix = n
        self.K = (n + 1) // 2
        self.omega = 1.0 / n

    def synth(self, a):
        return self.n * np.fft.irfft(a[:, 0] + 1j * a[:, 1], self.n)

    def adjoint(self, x):
        f = np.fft.rfft(x)
        return np.stack([f.real, f.imag], axis=1)

    def ell(self):
        return np.arange(self.K)

    def dot(self, a, b):
        w = np.full(self.K, 2.0)
        w[0] = 1.0
        return float(np.sum(w * (a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1])))


def dense_generic(T, cl, w, d):
    """Wiener filter over real parameters by probing T.synth with unit vectors (small problems)."""
    ell = T.ell()
    cols, prec = [], []
    for k in range(ell.size):
        if cl[ell[k]] <= 0:
            continue
        for part in (0, 1):
            if part == 1 and k == 0:
                continue
            cols.append((k, part))
            prec.append((1.0 if k == 0 else 2.0) / cl[ell[k]])
    Y = np.zeros((T.npix, len(cols)))
    for j, (k, part) in enumerate(cols):
        e = np.zeros((ell.size, 2))
        e[k, part] = 1.0
        Y[:, j] = T.synth(e)
    A = Y.T @ (w[:, None] * Y) + np.diag(prec)
    x = np.linalg.solve(A, Y.T @ (w * d))
    out = np.zeros((ell.size, 2))
    for j, (k, part) in enumerate(cols):
        out[k, part] = x[j]
    return out


def toy_problem(n=255, seed=3, homogeneous=False, masked=True):
    rng = np.random.default_rng(seed)
    T = Toy1D(n)
    k = np.arange(T.K, dtype=float)
    cl = np.where(k >= 1, 100.0 / (1.0 + k) ** 2, 0.0)
    a = np.zeros((T.K, 2))
    a[1:] = rng.standard_normal((T.K - 1, 2)) * np.sqrt(cl[1:] / 2)[:, None]
    sig = np.full(n, 0.3) if homogeneous else 0.3 * np.exp(rng.normal(0, 0.5, n))
    w = 1.0 / sig ** 2
    if masked:
        w[100:106] = 0.0
    d = T.synth(a) + sig * rng.standard_normal(n)
    d[w == 0] = 0.0
    return T, cl, w, d


# --------------------------------------------------------------------------
# schedule
# --------------------------------------------------------------------------
def test_level_schedule_rules():
    alpha, sigma, beta = 2.0, 100.0, 0.75
    cl = np.array([0.0, 0.0, 5.0, 3.0, 1.0])
    xs = dm.level_schedule(alpha, sigma, cl, beta)
    assert xs[0] == pytest.approx(alpha + sigma * beta * 5.0)
    assert xs[-1] == alpha
    for a_, b_ in zip(xs[:-2], xs[1:-1]):
        assert b_ == pytest.approx(beta * a_)
    assert beta * xs[-2] <= alpha < xs[-2]
    assert dm.level_schedule(alpha, sigma, np.zeros(3), beta) == [alpha]
    # Heaviside truncation: modes with C_l <= mu are switched off (f = 0)
    mu, f, li = dm.level_params(alpha + sigma * 3.0, alpha, sigma, cl)
    assert mu == pytest.approx(3.0)
    assert li == 2 and f[3] == 0.0 and f[4] == 0.0 and f[2] > 0.0


# --------------------------------------------------------------------------
# dense solve: the plain definition
# --------------------------------------------------------------------------
def test_dense_solution_satisfies_wf_equation_with_independent_basis():
    """(C^-1 + Y^H W Y) a = Y^H W d checked with Y built from scipy's Y_lm."""
    p, T, d, w = sphere_problem(nside=4, lmax=8)
    a = dense.wiener_dense(4, p.lmax, p.cl, w, d)
    th, ph = oracle.pixel_angles(4)
    lmax = p.lmax
    # complex synthesis matrix over (l, m >= 0) with the real-field convention
    s = np.zeros(th.size)
    grads = {}
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            k = oracle.alm_index(l, m, lmax)
            Y = sph_harm_y(l, m, th, ph)
            c = a[k, 0] + 1j * a[k, 1]
            s += (c * Y).real if m == 0 else 2 * (c * Y).real
            grads[k] = Y
    r = w * (d - s)
    for k, Y in grads.items():
        l = oracle.ell_of_index(lmax)[k]
        if p.cl[l] <= 0:
            assert a[k, 0] == 0 and a[k, 1] == 0
            continue
        g = np.sum(r * np.conj(Y))
        lhs = (a[k, 0] + 1j * a[k, 1]) / p.cl[l]
        assert abs(lhs - g) <= 1e-10 * (abs(g) + 1e-3)


def test_dense_wf_residual_and_chi2_minimum():
    p, T, d, w = sphere_problem(nside=8)
    a = dense.wiener_dense(8, p.lmax, p.cl, w, d)
    assert dm.wf_residual(T, a, d, w, p.cl) < 1e-12
    c0 = dm.chi2(T, a, d, w, p.cl)
    rng = np.random.default_rng(0)
    act = p.cl[oracle.ell_of_index(p.lmax)] > 0
    for _ in range(3):
        delta = rng.standard_normal(a.shape) * 1e-3 * act[:, None]
        delta[:p.lmax + 1, 1] = 0.0
        assert dm.chi2(T, a + delta, d, w, p.cl) > c0


# --------------------------------------------------------------------------
# the iteration against its fixed points
# --------------------------------------------------------------------------
def test_dm_converges_to_dense_wf_nside8():
    p, T, d, w = sphere_problem(nside=8)
    res = dm.solve(T, d, w, p.cl, eps_final=1e-12, eps_coarse=1e-4)
    ref = dense.wiener_dense(8, p.lmax, p.cl, w, d)
    assert res.converged
    assert rel(res.alm, ref) < 1e-8
    assert rel(res.map, T.synth(ref)) < 1e-8
    assert dm.wf_residual(T, res.alm, d, w, p.cl) < 1e-8
    assert res.xis[-1] == res.alpha
    assert all(np.diff(res.ell_iters) >= 0)


@pytest.mark.slow
def test_dm_config1_full_size():
    """Configuration 1 (Nside 16, lmax 32) against the dense Wiener filter."""
    p, T, d, w = sphere_problem(nside=16)
    res = dm.solve(T, d, w, p.cl, eps_final=1e-10, eps_coarse=1e-4)
    ref = dense.wiener_dense(16, p.lmax, p.cl, w, d)
    assert rel(res.alm, ref) < 1e-6


def test_level_fixed_point_matches_dense():
    """At fixed xi the iteration converges to (S_bar^-1 + Y^H (N + xi - alpha)^-1 Y) a = Y^H (N + xi - alpha)^-1 d."""
    p, T, d, w = sphere_problem(nside=8)
    alpha = dm.alpha_of(w)
    sigma = 1.0 / T.omega
    xis = dm.level_schedule(alpha, sigma, p.cl, 0.75)
    xi = xis[len(xis) // 2]
    # direct single-level run
    mu, f, _ = dm.level_params(xi, alpha, sigma, p.cl)
    c = dm.pixel_coeff(xi, alpha, w)
    a = np.zeros((oracle.n_alm(p.lmax), 2))
    r = np.where(w > 0, d, 0.0)
    s_prev = np.zeros_like(d)
    for _ in range(20000):
        a, s, r, num, den = dm.iterate(T, a, r, f[T.ell()], c, d, s_prev)
        s_prev = s
        if dm.cauchy_ratio(num, den) < 1e-14:
            break
    ref = dense.level_fixed_point(8, p.lmax, p.cl, w, d, xi, alpha, sigma)
    assert rel(a, ref) < 1e-10


def test_truncation_is_exact():
    """Modes above l_iter stay exactly zero through a level (f_l = 0 there)."""
    p, T, d, w = sphere_problem(nside=8)
    res = dm.solve(T, d, w, p.cl, eps_final=1e-3, eps_coarse=1e-3, replay=None)
    alpha = res.alpha
    sigma = 1.0 / T.omega
    xi = res.xis[3]
    mu, f, li = dm.level_params(xi, alpha, sigma, p.cl)
    a = np.zeros((oracle.n_alm(p.lmax), 2))
    a, s, r, *_ = dm.iterate(T, a, np.where(w > 0, d, 0.0), f[T.ell()], dm.pixel_coeff(xi, alpha, w), d,
                             np.zeros_like(d))
    assert li < p.lmax
    assert np.all(a[oracle.ell_of_index(p.lmax) > li] == 0.0)


# --------------------------------------------------------------------------
# exact-transform toy: the paper's algebra verbatim
# --------------------------------------------------------------------------
def test_toy_converges_to_wf():
    T, cl, w, d = toy_problem()
    res = dm.solve(T, d, w, cl, eps_final=1e-12, eps_coarse=1e-6, max_iter=100000)
    ref = dense_generic(T, cl, w, d)
    assert res.converged
    assert rel(res.alm, ref) < 1e-7


def test_toy_homogeneous_noise_one_step_per_level():
    """N = alpha 1: N_bar = 0 so t = d and each level is solved exactly by its first step."""
    T, cl, w, d = toy_problem(homogeneous=True, masked=False)
    res = dm.solve(T, d, w, cl, eps_final=1e-14, eps_coarse=1e-14)
    assert all(n <= 2 for n in res.iters_per_level)
    assert rel(res.alm, dense_generic(T, cl, w, d)) < 1e-12


def test_toy_error_contracts_within_a_level():
    """|eps_{i+1}| < |eps_i| inside one level (paper, dual residual recursion), down to rounding."""
    T, cl, w, d = toy_problem()
    alpha = dm.alpha_of(w)
    sigma = 1.0 / T.omega
    xs = dm.level_schedule(alpha, sigma, cl, 0.75)
    for lev in (6, len(xs) - 1):
        xi = xs[lev]
        mu, f, _ = dm.level_params(xi, alpha, sigma, cl)
        sbar = np.where(cl - mu > 0, cl - mu, 0.0)
        ref = dense_generic(T, sbar, w / (1 + (xi - alpha) * w), d)
        c = dm.pixel_coeff(xi, alpha, w)
        a = np.zeros((T.K, 2))
        r = np.where(w > 0, d, 0.0)
        s_prev = np.zeros(T.n)
        errs = []
        for _ in range(60):
            a, s, r, *_ = dm.iterate(T, a, r, f[T.ell()], c, d, s_prev)
            s_prev = s
            errs.append(rel(a, ref))
        live = [e for e in errs if e > 1e-12]
        assert len(live) >= 5
        assert all(b < a_ for a_, b in zip(live[:-1], live[1:]))


def test_beta_half_needs_fewer_iterations():
    """Paper Section 4: beta = 1/2 instead of 3/4 reduces the iteration count at eps = 1e-6."""
    p, T, d, w = sphere_problem(nside=8)
    n34 = dm.solve(T, d, w, p.cl, beta=0.75, eps_final=1e-6, eps_coarse=1e-6).n_iter
    n12 = dm.solve(T, d, w, p.cl, beta=0.5, eps_final=1e-6, eps_coarse=1e-6).n_iter
    assert n12 < n34


# --------------------------------------------------------------------------
# planted mistakes: the pins above must catch them
# --------------------------------------------------------------------------
def test_planted_N_instead_of_Nbar_is_caught(monkeypatch):
    """With N^-1 (as the printed pixel step reads) the fixed point is not the Wiener filter."""
    T, cl, w, d = toy_problem()
    monkeypatch.setattr(dm, "pixel_coeff", lambda xi, alpha, w_: xi * w_ / (1.0 + xi * w_))
    res = dm.solve(T, d, w, cl, eps_final=1e-12, eps_coarse=1e-6, max_iter=100000)
    assert rel(res.alm, dense_generic(T, cl, w, d)) > 1e-4


def test_planted_missing_sigma_is_caught(monkeypatch):
    T, cl, w, d = toy_problem()
    orig = dm.level_params

    def wrong(xi, alpha, sigma, cl_):
        mu, f, li = orig(xi, alpha, sigma, cl_)
        sbar = np.where(cl_ - mu > 0, cl_ - mu, 0.0)
        return mu, sbar / (sbar + xi), li

    monkeypatch.setattr(dm, "level_params", wrong)
    res = dm.solve(T, d, w, cl, eps_final=1e-12, eps_coarse=1e-6, max_iter=20000)
    assert rel(res.alm, dense_generic(T, cl, w, d)) > 1e-4


def test_literal_harmonic_step_is_biased_on_healpix(monkeypatch):
    """a = f Omega Y^H t (no residual) drifts from the Wiener filter when Omega Y^H Y != 1."""
    p, T, d, w = sphere_problem(nside=8)

    def literal(T_, a, r, f_alm, c, d_, s_prev):
        t = T_.synth(a) + r if a.any() else r
        a = f_alm[:, None] * (T_.omega * T_.adjoint(t))
        s = T_.synth(a)
        return a, s, c * (d_ - s), float(np.sum((s - s_prev) ** 2)), float(np.sum(s * s))

    ref = dense.wiener_dense(8, p.lmax, p.cl, w, d)
    good = dm.solve(T, d, w, p.cl, eps_final=1e-10, eps_coarse=1e-4)
    monkeypatch.setattr(dm, "iterate", literal)
    bad = dm.solve(T, d, w, p.cl, eps_final=1e-10, eps_coarse=1e-4)
    assert rel(good.alm, ref) < 1e-6
    assert rel(bad.alm, ref) > 1e-3


# --------------------------------------------------------------------------
# the warm-start branch and the reported residual, pinned independently
# --------------------------------------------------------------------------
def test_warm_start_branch_stays_at_and_converges_to_dense_wf():
    """The solve started at xi = alpha from a given a_lm (Algorithm 2's loop
    entered at its last level).  Started at the dense Wiener filter it stays
    there: the WF is the fixed point of the residual-form step at mu = 0, so the
    first iterate equals the start and the first Cauchy ratio is at rounding
    level.  Started 20% away (in every active mode) it converges to the dense
    solution."""
    p, T, d, w = sphere_problem(nside=8)
    ref = dense.wiener_dense(8, p.lmax, p.cl, w, d)
    stay = dm.solve(T, d, w, p.cl, start_final=True, alm0=ref, replay=[1])
    assert stay.n_iter == 1
    assert rel(stay.alm, ref) < 1e-12
    assert stay.ratios[0] < 1e-12
    rng = np.random.default_rng(8)
    act = p.cl[oracle.ell_of_index(p.lmax)] > 0
    start = ref + 0.2 * np.abs(ref).mean() * rng.standard_normal(ref.shape) * act[:, None]
    start[:p.lmax + 1, 1] = 0.0
    assert rel(start, ref) > 0.1
    res = dm.solve(T, d, w, p.cl, start_final=True, alm0=start, eps_final=1e-13,
                   max_iter=200000)
    assert res.converged and len(res.iters_per_level) == 1
    assert rel(res.alm, ref) < 1e-8
    assert rel(res.map, T.synth(ref)) < 1e-8


def test_wf_residual_matches_independent_scipy_basis():
    """||A x - y|| / ||y|| (A = 1 + C^1/2 Y^H W Y C^1/2, x = C^-1/2 a,
    y = C^1/2 Y^H W d) of a perturbed a_lm, built here from scipy's Y_lm with
    explicit sums over pixels and modes, norms counting m > 0 twice; the
    oracle's value must agree."""
    nside, lmax = 4, 8
    p, T, d, w = sphere_problem(nside=nside, lmax=lmax)
    rng = np.random.default_rng(4)
    a = dense.wiener_dense(nside, lmax, p.cl, w, d)
    a = a + 0.3 * np.abs(a).mean() * rng.standard_normal(a.shape)
    a[:lmax + 1, 1] = 0.0
    th, ph = oracle.pixel_angles(nside)
    Y, s = {}, np.zeros(th.size)
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            k = oracle.alm_index(l, m, lmax)
            Y[k] = (l, m, sph_harm_y(l, m, th, ph))
            c = a[k, 0] + 1j * a[k, 1]
            s += (c * Y[k][2]).real * (1.0 if m == 0 else 2.0)
    r2 = y2 = 0.0
    for k, (l, m, Ylm) in Y.items():
        if p.cl[l] <= 0.0:
            continue
        sq = math.sqrt(p.cl[l])
        g = np.sum(w * (d - s) * np.conj(Ylm))
        yv = sq * np.sum(w * d * np.conj(Ylm))
        res = (a[k, 0] + 1j * a[k, 1]) / sq - sq * g
        wt = 1.0 if m == 0 else 2.0
        r2 += wt * abs(res) ** 2
        y2 += wt * abs(yv) ** 2
    want = math.sqrt(r2 / y2)
    assert want > 1e-3  # a perturbed point, far from the zero at the solution
    assert dm.wf_residual(T, a, d, w, p.cl) == pytest.approx(want, rel=1e-10)
