"""GPU path (through the C ABI) against the CPU oracle, element by element.

Sizes span one to many 64-lane chunks of ring pairs with ragged tails, lmax up
to 3N-1 (aliasing in the polar rings), Nside 1 and 2.  FP64 bar: relative L2
1e-12 for single transforms and 1e-10 for iterations and solves (the oracle
sums in a different order; rounding differences grow with the iteration).
"""
import numpy as np
import pytest

import dmwf_inputs as inp
import oracle
from oracle import dm
from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu

SIZES = [(1, 0), (1, 2), (2, 5), (4, 8), (4, 11), (8, 16), (8, 23), (16, 32), (16, 47),
         (32, 64), (64, 128), (64, 191)]


def _plan(nside, lmax, nmaps=1):
    from paper_1702_08852_amd import Plan
    return Plan(nside, lmax, nmaps=nmaps, device=device())


@pytest.mark.parametrize("nside,lmax", SIZES)
def test_alm2map(nside, lmax):
    dev = device()
    a = inp.random_alm(lmax, 100 + nside + lmax)
    ref = oracle.alm2map(a, nside, lmax)
    got = _plan(nside, lmax).alm2map(to_dev(a, dev)).cpu().numpy()
    assert rel(got, ref) < 1e-12


@pytest.mark.parametrize("nside,lmax", SIZES)
def test_adjoint(nside, lmax):
    dev = device()
    mp = inp.random_map(nside, 200 + nside + lmax)
    ref = oracle.adjoint(mp, nside, lmax)
    plan = _plan(nside, lmax)
    got = plan.adjoint(to_dev(mp, dev)).cpu().numpy()
    assert rel(got, ref) < 1e-12
    assert np.all(got[:lmax + 1, 1] == 0.0)
    got2 = plan.adjoint(to_dev(mp, dev), scale_by_pixel_area=True).cpu().numpy()
    assert rel(got2, ref * (4 * np.pi / mp.size)) < 1e-12


def test_alm2map_ignores_imaginary_m0():
    dev = device()
    nside, lmax = 8, 16
    a = inp.random_alm(lmax, 5)
    b = a.copy()
    b[:lmax + 1, 1] = 123.0
    plan = _plan(nside, lmax)
    np.testing.assert_array_equal(plan.alm2map(to_dev(a, dev)).cpu().numpy(),
                                  plan.alm2map(to_dev(b, dev)).cpu().numpy())


def test_multi_map_transforms():
    dev = device()
    nside, lmax, nm = 8, 16, 3
    a = np.stack([inp.random_alm(lmax, 300 + k) for k in range(nm)])
    plan = _plan(nside, lmax, nmaps=nm)
    got = plan.alm2map(to_dev(a, dev)).cpu().numpy()
    for k in range(nm):
        assert rel(got[k], oracle.alm2map(a[k], nside, lmax)) < 1e-12


def _cfg1(nside):
    p = inp.make_problem("cfg1", nside=nside)
    T = oracle.SphereTransforms(nside, p.lmax)
    d = p.data_map(T.synth(p.alm_true))
    return p, T, d, p.ninv


@pytest.mark.parametrize("nside,level", [(8, 3), (16, 10), (16, 0)])
def test_dm_iterate_matches_oracle_step_by_step(nside, level):
    import torch
    dev = device()
    p, T, d, w = _cfg1(nside)
    alpha = dm.alpha_of(w)
    sigma = 1.0 / T.omega
    xi = dm.level_schedule(alpha, sigma, p.cl, 0.75)[level]
    mu, f, _ = dm.level_params(xi, alpha, sigma, p.cl)
    c = dm.pixel_coeff(xi, alpha, w)
    plan = _plan(nside, p.lmax)
    cl_t, d_t, w_t = to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev)
    a_t = torch.zeros((oracle.n_alm(p.lmax), 2), dtype=torch.float64, device=dev)
    s_t = torch.full((12 * nside * nside,), 7.0, dtype=torch.float64, device=dev)
    c2 = torch.zeros(2, dtype=torch.float64, device=dev)
    a = np.zeros((oracle.n_alm(p.lmax), 2))
    r = np.where(w > 0, d, 0.0)
    s_prev = np.zeros_like(d)
    for it in range(6):
        plan.dm_iterate(xi, alpha, cl_t, d_t, w_t, a_t, s_t, c2, first=(it == 0))
        a, s, r, num, den = dm.iterate(T, a, r, f[T.ell()], c, d, s_prev)
        s_prev = s
        assert rel(a_t.cpu().numpy(), a) < 1e-11
        assert rel(s_t.cpu().numpy(), s) < 1e-11
        cc = c2.cpu().numpy()
        assert cc[0] == pytest.approx(num, rel=1e-9, abs=1e-12 * den)
        assert cc[1] == pytest.approx(den, rel=1e-11)


@pytest.mark.parametrize("nside", [8, 16])
def test_solve_replayed_matches_oracle(nside):
    dev = device()
    p, T, d, w = _cfg1(nside)
    plan = _plan(nside, p.lmax)
    alm, smap, st = plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev),
                               eps_final=1e-8, eps_coarse=1e-4, want_residual=True)
    assert st.status == 0
    ref = dm.solve(T, d, w, p.cl, eps_final=1e-8, eps_coarse=1e-4, replay=st.iters_per_level)
    np.testing.assert_allclose(st.xi_per_level, ref.xis, rtol=1e-15)
    assert st.lmax_per_level == ref.ell_iters
    assert st.alpha == pytest.approx(ref.alpha, rel=1e-15)
    assert rel(alm.cpu().numpy(), ref.alm) < 1e-10
    assert rel(smap.cpu().numpy(), ref.map) < 1e-10
    assert st.final_cauchy < 1e-8
    assert st.wf_residual == pytest.approx(dm.wf_residual(T, ref.alm, d, w, p.cl), rel=1e-6)
    # the oracle's own stopping decisions land on the same iteration counts
    free = dm.solve(T, d, w, p.cl, eps_final=1e-8, eps_coarse=1e-4)
    assert abs(free.n_iter - st.n_iter) <= max(2, len(st.iters_per_level) // 4)


def test_solve_warm_start_final_level():
    dev = device()
    nside = 8
    p, T, d, w = _cfg1(nside)
    plan = _plan(nside, p.lmax)
    warm = dm.solve(T, d, w, p.cl, eps_final=1e-4, eps_coarse=1e-3).alm
    alm0 = to_dev(warm, dev)
    alm, smap, st = plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev), eps_final=1e-9,
                               start_final=True, alm=alm0)
    assert st.n_levels == 1
    ref = dm.solve(T, d, w, p.cl, start_final=True, alm0=warm, replay=st.iters_per_level)
    assert rel(alm.cpu().numpy(), ref.alm) < 1e-10


def test_solve_error_paths():
    import torch
    from paper_1702_08852_amd import DmwfError
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    nside = 4
    p, T, d, w = _cfg1(nside)
    plan = _plan(nside, p.lmax)
    cl_t, d_t, w_t = to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev)
    with pytest.raises(DmwfError) as e:
        plan.solve(cl_t, d_t, torch.zeros_like(w_t))
    assert e.value.status == b.ERR_INVALID_ARG
    bad = d.copy()
    bad[5] = np.nan
    with pytest.raises(DmwfError) as e:
        plan.solve(cl_t, to_dev(bad, dev), w_t)
    assert e.value.status == b.ERR_NONFINITE
    neg = w.copy()
    neg[3] = -1.0
    with pytest.raises(DmwfError) as e:
        plan.solve(cl_t, d_t, to_dev(neg, dev))
    assert e.value.status == b.ERR_NONFINITE
    with pytest.raises(DmwfError) as e:
        plan.solve(cl_t, d_t, w_t, beta=1.5)
    assert e.value.status == b.ERR_INVALID_ARG
    with pytest.raises(DmwfError) as e:
        plan.solve(cl_t, d_t, w_t, replay=[1, 2])
    assert e.value.status == b.ERR_INVALID_ARG
    _, _, st = plan.solve(cl_t, d_t, w_t, max_iter=3)
    assert st.status == b.ERR_NOT_CONVERGED and st.n_iter == 3
    # workspace too small
    import ctypes
    lib = b.load()
    out = torch.empty(12 * nside * nside, dtype=torch.float64, device=dev)
    alm = torch.zeros((oracle.n_alm(p.lmax), 2), dtype=torch.float64, device=dev)
    s = lib.dmwf_alm2map(plan._h, alm.data_ptr(), out.data_ptr(), plan.ws.data_ptr(),
                         plan.ws_bytes - 1, None)
    assert s == b.ERR_WORKSPACE
    s = lib.dmwf_dm_iterate(plan._h, ctypes.c_double(0.5), ctypes.c_double(1.0), cl_t.data_ptr(),
                            d_t.data_ptr(), w_t.data_ptr(), alm.data_ptr(), out.data_ptr(),
                            out.data_ptr(), 1, plan.ws.data_ptr(), plan.ws_bytes, None)
    assert s == b.ERR_INVALID_ARG


def test_solve_replays_oracle_schedule():
    """The device-side level control honours replayed per-level counts: the
    oracle decides its own stops, the GPU replays them and lands on the same
    iterate."""
    dev = device()
    nside = 8
    p, T, d, w = _cfg1(nside)
    ref = dm.solve(T, d, w, p.cl, eps_final=1e-9, eps_coarse=1e-4)
    plan = _plan(nside, p.lmax)
    alm, smap, st = plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev),
                               eps_final=1e-9, eps_coarse=1e-4, replay=ref.iters_per_level)
    assert st.status == 0
    assert st.iters_per_level == list(ref.iters_per_level)
    assert st.n_iter == ref.n_iter
    assert rel(alm.cpu().numpy(), ref.alm) < 1e-10
    assert rel(smap.cpu().numpy(), ref.map) < 1e-10


def test_solve_iteration_cap_inside_a_level():
    """A cap that falls in the middle of a level stops there: the counts of the
    levels run add up to the cap and the state is the oracle's after as many
    iterations."""
    dev = device()
    nside = 8
    p, T, d, w = _cfg1(nside)
    plan = _plan(nside, p.lmax)
    full = dm.solve(T, d, w, p.cl, eps_final=1e-8, eps_coarse=1e-4)
    cap = full.iters_per_level[0] + full.iters_per_level[1] + 2
    alm, smap, st = plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev),
                               eps_final=1e-8, eps_coarse=1e-4, max_iter=cap)
    from paper_1702_08852_amd import dmwf as b
    assert st.status == b.ERR_NOT_CONVERGED
    assert st.n_iter == cap and sum(st.iters_per_level) == cap
    # the oracle replays the completed levels and is cut by the same cap on the
    # last one (its count there is set beyond the cap)
    nrest = len(full.iters_per_level) - len(st.iters_per_level)
    replay = st.iters_per_level[:-1] + [st.iters_per_level[-1] + 1000] + [1] * nrest
    ref = dm.solve(T, d, w, p.cl, eps_final=1e-8, eps_coarse=1e-4, replay=replay, max_iter=cap)
    assert ref.n_iter == cap and not ref.converged
    assert rel(alm.cpu().numpy(), ref.alm) < 1e-10


def test_solve_two_maps_match_single_map_solves():
    """A plan with two maps (of different spectra, noise and masks) solves them
    together, each exactly as a single-map plan would."""
    import torch
    dev = device()
    nside = 8
    p, T, d, w = _cfg1(nside)
    d2 = np.roll(d, 37)
    w2 = np.roll(w, 37)
    cl2 = p.cl * 2.0
    single = _plan(nside, p.lmax)
    a1, s1, _ = single.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev), eps_final=1e-8)
    a1, s1 = a1.cpu().numpy(), s1.cpu().numpy()
    a2, s2, _ = single.solve(to_dev(cl2, dev), to_dev(d2, dev), to_dev(w2, dev), eps_final=1e-8)
    a2, s2 = a2.cpu().numpy(), s2.cpu().numpy()
    from paper_1702_08852_amd import Plan
    two = Plan(nside, p.lmax, nmaps=2, device=dev)
    cl_t = torch.tensor(np.stack([p.cl, cl2]), device=dev)
    alm, smap, _ = two.solve(cl_t, torch.tensor(np.stack([d, d2]), device=dev),
                             torch.tensor(np.stack([w, w2]), device=dev), eps_final=1e-8)
    alm, smap = alm.cpu().numpy(), smap.cpu().numpy()
    assert rel(alm[0], a1) < 1e-13 and rel(alm[1], a2) < 1e-13
    assert rel(smap[0], s1) < 1e-13 and rel(smap[1], s2) < 1e-13


def test_solve_rejects_schedules_beyond_the_level_table():
    """More cooling levels than the device level table holds is an argument
    error raised before any iteration runs."""
    from paper_1702_08852_amd import DmwfError
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    nside = 4
    p, T, d, w = _cfg1(nside)
    plan = _plan(nside, p.lmax)
    with pytest.raises(DmwfError) as e:
        plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev), beta=0.9999)
    assert e.value.status == b.ERR_INVALID_ARG


def test_solve_cap_on_a_level_switch_stops():
    """A cap that falls on the iteration that completes a level stops the
    solve there (not converged, exactly the cap), instead of entering the next
    level; likewise with several maps."""
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    nside = 8
    p, T, d, w = _cfg1(nside)
    plan = _plan(nside, p.lmax)
    cl_t, d_t, w_t = to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev)
    _, _, full = plan.solve(cl_t, d_t, w_t, eps_final=1e-8, eps_coarse=1e-4)
    for nlev in (1, 3):
        cap = sum(full.iters_per_level[:nlev])
        _, _, st = plan.solve(cl_t, d_t, w_t, eps_final=1e-8, eps_coarse=1e-4, max_iter=cap)
        assert st.status == b.ERR_NOT_CONVERGED and st.n_iter == cap
        assert st.iters_per_level == full.iters_per_level[:nlev]
    # the last level completed on the capped iteration is a convergence
    _, _, st = plan.solve(cl_t, d_t, w_t, eps_final=1e-8, eps_coarse=1e-4, max_iter=full.n_iter)
    assert st.status == b.OK and st.n_iter == full.n_iter
    two = _plan(nside, p.lmax, nmaps=2)
    import torch
    cap = full.iters_per_level[0]
    _, _, sts = two.solve(torch.stack([cl_t, cl_t]), torch.stack([d_t, d_t]),
                          torch.stack([w_t, w_t]), eps_final=1e-8, eps_coarse=1e-4, max_iter=cap)
    assert all(s.status == b.ERR_NOT_CONVERGED and s.n_iter == cap for s in sts)
