"""Degenerate inputs of the method on the GPU, through the C ABI, against the
oracle: zero data, no mask with homogeneous noise (N = alpha everywhere, so
N_bar = 0 and the pixel coefficient is 1 at xi = alpha), a single observed
pixel, and a spectrum that vanishes above half the band (Algorithm 2 with the
truncation of Appendix B).  Every GPU solve is compared with the oracle
replaying the GPU's per-level iteration counts (relative L2 1e-10)."""
import numpy as np
import pytest

import dmwf_inputs as inp
import oracle
from oracle import dense, dm
from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu

NSIDE = 8


def _problem():
    p = inp.make_problem("cfg1", nside=NSIDE)
    T = oracle.SphereTransforms(NSIDE, p.lmax)
    return p, T


def _gpu_solve(lmax, cl, d, w, eps_final=1e-9):
    from paper_1702_08852_amd import Plan
    dev = device()
    plan = Plan(NSIDE, lmax, device=dev)
    alm, smap, st = plan.solve(to_dev(cl, dev), to_dev(d, dev), to_dev(w, dev),
                               eps_final=eps_final, eps_coarse=1e-4, want_residual=True)
    assert st.status == 0
    return alm.cpu().numpy(), smap.cpu().numpy(), st


def _replayed(T, cl, d, w, st, eps_final=1e-9):
    return dm.solve(T, d, w, cl, eps_final=eps_final, eps_coarse=1e-4,
                    replay=st.iters_per_level)


def test_zero_data_gives_the_zero_solution_in_one_iteration_per_level():
    p, T = _problem()
    d = np.zeros(12 * NSIDE * NSIDE)
    alm, smap, st = _gpu_solve(p.lmax, p.cl, d, p.ninv)
    # r = 0 on the first iteration, so a = s = 0 and the Cauchy ratio is 0 / 0,
    # which counts as converged: one iteration on every level
    assert not alm.any() and not smap.any()
    free = dm.solve(T, d, p.ninv, p.cl, eps_final=1e-9, eps_coarse=1e-4)
    assert st.iters_per_level == list(free.iters_per_level)
    assert all(n == 1 for n in st.iters_per_level)
    assert st.final_cauchy == 0.0


def test_unmasked_homogeneous_noise():
    p, T = _problem()
    sigma = 0.5
    rng = np.random.default_rng(1702)
    w = np.full(12 * NSIDE * NSIDE, 1.0 / sigma**2)
    d = T.synth(p.alm_true) + sigma * rng.standard_normal(w.size)
    alm, smap, st = _gpu_solve(p.lmax, p.cl, d, w)
    assert st.alpha == pytest.approx(sigma**2, rel=1e-15)
    ref = _replayed(T, p.cl, d, w, st)
    assert rel(alm, ref.alm) < 1e-10
    assert rel(smap, ref.map) < 1e-10
    # the fixed point of the last level is the Wiener filter itself
    a_wf = dense.wiener_dense(NSIDE, p.lmax, p.cl, w, d)
    assert rel(alm, a_wf) < 1e-6
    assert st.wf_residual < 1e-6


def test_single_observed_pixel():
    p, T = _problem()
    w = np.zeros(12 * NSIDE * NSIDE)
    pix = 6 * NSIDE * NSIDE + 3  # on the equator
    w[pix] = 4.0
    d = T.synth(p.alm_true) + 0.5 * np.random.default_rng(5).standard_normal(w.size)
    alm, smap, st = _gpu_solve(p.lmax, p.cl, d, w)
    assert st.alpha == pytest.approx(0.25, rel=1e-15)
    ref = _replayed(T, p.cl, d, w, st)
    assert rel(alm, ref.alm) < 1e-10
    assert rel(smap, ref.map) < 1e-10
    a_wf = dense.wiener_dense(NSIDE, p.lmax, p.cl, w, d)
    assert rel(alm, a_wf) < 1e-6


def test_spectrum_vanishing_above_half_the_band():
    p, T = _problem()
    cl = np.array(p.cl, dtype=np.float64)
    half = p.lmax // 2
    cl[half + 1:] = 0.0
    d = p.data_map(T.synth(p.alm_true))
    alm, smap, st = _gpu_solve(p.lmax, cl, d, p.ninv)
    # modes with C_l = 0 are never active: l_iter <= lmax / 2 on every level
    # and their coefficients stay exactly zero
    assert max(st.lmax_per_level) <= half
    ell = T.ell()
    assert not alm[ell > half].any()
    ref = _replayed(T, cl, d, p.ninv, st)
    assert rel(alm, ref.alm) < 1e-10
    assert rel(smap, ref.map) < 1e-10
