"""Batched solves on the GPU: the maps of one plan advance together, one launch
per stage for all of them, with the Legendre recurrence shared by the maps of
a wave and a level control of its own per map (each map has its own alpha,
schedule and stopping point).

Each map of a batch must come out bit for bit as a single-map plan computes
it (the per-map arithmetic is the same, in the same order), and within the
FP64 parity bar of the oracle replaying that map's per-level counts.  The
maps are members of the batched workload's recipe (own mask, noise level and
noise modulation per map) at sizes the oracle finishes in seconds.
"""
import numpy as np
import pytest

import dmwf_inputs as inp
import oracle
from oracle import dm
from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu


def _members(nside, n, first=0):
    ps = [inp.make_problem("cfg4", nside=nside, index=first + k) for k in range(n)]
    T = oracle.SphereTransforms(nside, ps[0].lmax)
    ds = [p.data_map(T.synth(p.alm_true)) for p in ps]
    return ps, T, ds


def _stack(arrs, dev):
    import torch
    return torch.tensor(np.stack(arrs), device=dev)


def torch_tensor(a, dev):
    import torch
    return torch.tensor(a, device=dev)


def _plan(nside, lmax, nmaps):
    from paper_1702_08852_amd import Plan
    return Plan(nside, lmax, nmaps=nmaps, device=device())


@pytest.mark.parametrize("nside,nmaps", [(4, 2), (8, 3), (8, 5), (16, 4)])
def test_batched_solve_equals_single_map_solves(nside, nmaps):
    dev = device()
    ps, T, ds = _members(nside, nmaps)
    lmax = ps[0].lmax
    batch = _plan(nside, lmax, nmaps)
    alm, smap, sts = batch.solve(_stack([p.cl for p in ps], dev), _stack(ds, dev),
                                 _stack([p.ninv for p in ps], dev), eps_final=1e-8)
    alm, smap = alm.cpu().numpy(), smap.cpu().numpy()
    assert len(sts) == nmaps
    single = _plan(nside, lmax, 1)
    counts = set()
    for k, p in enumerate(ps):
        a1, s1, st1 = single.solve(to_dev(p.cl, dev), to_dev(ds[k], dev), to_dev(p.ninv, dev),
                                   eps_final=1e-8)
        assert sts[k].status == 0 and st1.status == 0
        assert sts[k].iters_per_level == st1.iters_per_level
        assert sts[k].alpha == st1.alpha and sts[k].final_cauchy == st1.final_cauchy
        np.testing.assert_array_equal(alm[k], a1.cpu().numpy())
        np.testing.assert_array_equal(smap[k], s1.cpu().numpy())
        counts.add(sts[k].n_iter)
    # the maps stop at different iterations: the per-map control is exercised
    assert len(counts) > 1


def test_batched_solve_matches_oracle_per_map():
    dev = device()
    nside, nmaps = 8, 3
    ps, T, ds = _members(nside, nmaps, first=10)
    batch = _plan(nside, ps[0].lmax, nmaps)
    alm, smap, sts = batch.solve(_stack([p.cl for p in ps], dev), _stack(ds, dev),
                                 _stack([p.ninv for p in ps], dev), eps_final=1e-8,
                                 eps_coarse=1e-4, want_residual=True)
    alm, smap = alm.cpu().numpy(), smap.cpu().numpy()
    for k, p in enumerate(ps):
        ref = dm.solve(T, ds[k], p.ninv, p.cl, eps_final=1e-8, eps_coarse=1e-4,
                       replay=sts[k].iters_per_level)
        np.testing.assert_allclose(sts[k].xi_per_level, ref.xis, rtol=1e-15)
        assert sts[k].lmax_per_level == ref.ell_iters
        assert rel(alm[k], ref.alm) < 1e-10
        assert rel(smap[k], ref.map) < 1e-10
        assert sts[k].wf_residual == pytest.approx(
            dm.wf_residual(T, ref.alm, ds[k], p.ninv, p.cl), rel=1e-6)
    # the residual entry point gives every map's, as the solve reported them
    res = batch.wf_residual(_stack([p.cl for p in ps], dev), _stack(ds, dev),
                            _stack([p.ninv for p in ps], dev), torch_tensor(alm, dev))
    assert res == [s.wf_residual for s in sts]


def test_batched_warm_start_equals_single_map():
    dev = device()
    nside, nmaps = 8, 3
    ps, T, ds = _members(nside, nmaps, first=20)
    lmax = ps[0].lmax
    warm = [dm.solve(T, ds[k], p.ninv, p.cl, eps_final=1e-4, eps_coarse=1e-3).alm
            for k, p in enumerate(ps)]
    batch = _plan(nside, lmax, nmaps)
    alm, _, sts = batch.solve(_stack([p.cl for p in ps], dev), _stack(ds, dev),
                              _stack([p.ninv for p in ps], dev), eps_final=1e-9,
                              start_final=True, alm=_stack(warm, dev))
    single = _plan(nside, lmax, 1)
    for k, p in enumerate(ps):
        assert sts[k].n_levels == 1
        a1, _, _ = single.solve(to_dev(p.cl, dev), to_dev(ds[k], dev), to_dev(p.ninv, dev),
                                eps_final=1e-9, start_final=True, alm=to_dev(warm[k], dev))
        np.testing.assert_array_equal(alm[k].cpu().numpy(), a1.cpu().numpy())


@pytest.mark.parametrize("nside,lmax,nmaps", [(16, 40, 5), (8, 23, 3), (2, 5, 9), (32, 64, 8)])
def test_batched_transforms_match_oracle(nside, lmax, nmaps):
    """Batched synthesis and adjoint, every map against the oracle: lmax up to
    3 Nside - 1 (aliasing in the polar rings), map counts that leave the last
    map group of a wave partly empty, and Nside 2."""
    dev = device()
    a = [inp.random_alm(lmax, 400 + k) for k in range(nmaps)]
    mp = [inp.random_map(nside, 500 + k) for k in range(nmaps)]
    plan = _plan(nside, lmax, nmaps)
    plan.autotune()
    syn = plan.alm2map(_stack(a, dev)).cpu().numpy()
    adj = plan.adjoint(_stack(mp, dev)).cpu().numpy()
    for k in range(nmaps):
        assert rel(syn[k], oracle.alm2map(a[k], nside, lmax)) < 1e-12
        assert rel(adj[k], oracle.adjoint(mp[k], nside, lmax)) < 1e-12


def test_batched_solve_names_the_bad_map():
    from paper_1702_08852_amd import DmwfError
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    nside, nmaps = 4, 3
    ps, T, ds = _members(nside, nmaps)
    ds[1] = ds[1].copy()
    ds[1][7] = np.inf
    batch = _plan(nside, ps[0].lmax, nmaps)
    with pytest.raises(DmwfError) as e:
        batch.solve(_stack([p.cl for p in ps], dev), _stack(ds, dev),
                    _stack([p.ninv for p in ps], dev))
    assert e.value.status == b.ERR_NONFINITE
    assert "map 1" in str(e.value)


def test_every_legendre_tile_gives_the_same_result():
    """Every synthesis tile, and the maps per wave of the analysis, compute each
    map's sums in the same order: the maps come out bit for bit alike; the
    analysis ring pairs per lane differ in the order of the ring-pair sums only
    (rounding)."""
    dev = device()
    nside, lmax, nmaps = 16, 32, 5
    a = _stack([inp.random_alm(lmax, 600 + k) for k in range(nmaps)], dev)
    mp = _stack([inp.random_map(nside, 700 + k) for k in range(nmaps)], dev)
    plan = _plan(nside, lmax, nmaps)
    ref_syn = ref_adj = None
    for k in (1, 2):
        for mb in (1, 2, 4, 8):
            plan.set_tiles(k, mb, 8)
            got = plan.alm2map(a).cpu().numpy()
            if ref_syn is None:
                ref_syn = got
            np.testing.assert_array_equal(got, ref_syn)
    for ak in (4, 8):
        plan.set_tiles(2, 1, ak, 1)
        got = plan.adjoint(mp).cpu().numpy()
        plan.set_tiles(2, 1, ak, 2)
        np.testing.assert_array_equal(plan.adjoint(mp).cpu().numpy(), got)
        if ref_adj is None:
            ref_adj = got
        assert rel(got, ref_adj) < 1e-14
    for k in range(nmaps):
        ref = oracle.alm2map(a[k].cpu().numpy(), nside, lmax)
        assert rel(ref_syn[k], ref) < 1e-12
    (sk, smb, ak, amb), times = plan.autotune()
    assert sk in (1, 2) and smb in (1, 2, 4, 8) and ak in (4, 8) and amb in (1, 2)
    assert "syn2x1" in times and "ana8x1" in times and "ana4x2" in times
    np.testing.assert_array_equal(plan.alm2map(a).cpu().numpy(), ref_syn)


def test_set_tiles_rejects_bad_values():
    from paper_1702_08852_amd import DmwfError
    plan = _plan(512, 64, 1)
    for bad in ((3, 1, 8, 1), (2, 3, 8, 1), (2, 1, 2, 1), (2, 1, 4, 1),   # 4 per lane needs nside <= 256
                (2, 1, 8, 4)):
        with pytest.raises(DmwfError):
            plan.set_tiles(*bad)


def test_batched_solve_argument_errors_name_the_map():
    """A map with every pixel masked, and a replay list that fits some maps'
    schedules but not another's, are argument errors naming the map; nothing
    runs."""
    from paper_1702_08852_amd import DmwfError
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    nside, nmaps = 4, 3
    ps, T, ds = _members(nside, nmaps)
    batch = _plan(nside, ps[0].lmax, nmaps)
    cl, d = _stack([p.cl for p in ps], dev), _stack(ds, dev)
    w = [p.ninv for p in ps]
    w_bad = list(w)
    w_bad[2] = np.zeros_like(w[2])
    with pytest.raises(DmwfError) as e:
        batch.solve(cl, d, _stack(w_bad, dev))
    assert e.value.status == b.ERR_INVALID_ARG and "map 2" in str(e.value)
    # the maps' schedules differ in length when their alpha differ enough
    cl2 = [p.cl for p in ps]
    cl2[1] = cl2[1] * 1e6
    nlev = [len(dm.level_schedule(dm.alpha_of(w[k]), 1.0 / T.omega, cl2[k], 0.75))
            for k in range(nmaps)]
    assert len(set(nlev)) > 1
    with pytest.raises(DmwfError) as e:
        batch.solve(_stack(cl2, dev), d, _stack(w, dev), replay=[1] * nlev[0])
    assert e.value.status == b.ERR_INVALID_ARG and "map" in str(e.value)


def test_batched_iteration_cap_stops_every_map():
    """A cap below every map's need stops each map at the cap; the statuses
    report it and the outputs hold each map's iterate after that many
    iterations, as a one-map plan computes it."""
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    nside, nmaps = 8, 3
    ps, T, ds = _members(nside, nmaps, first=30)
    lmax = ps[0].lmax
    batch = _plan(nside, lmax, nmaps)
    alm, smap, sts = batch.solve(_stack([p.cl for p in ps], dev), _stack(ds, dev),
                                 _stack([p.ninv for p in ps], dev), eps_final=1e-8, max_iter=17)
    single = _plan(nside, lmax, 1)
    for k, p in enumerate(ps):
        assert sts[k].status == b.ERR_NOT_CONVERGED and sts[k].n_iter == 17
        a1, s1, st1 = single.solve(to_dev(p.cl, dev), to_dev(ds[k], dev), to_dev(p.ninv, dev),
                                   eps_final=1e-8, max_iter=17)
        np.testing.assert_array_equal(alm[k].cpu().numpy(), a1.cpu().numpy())
        np.testing.assert_array_equal(smap[k].cpu().numpy(), s1.cpu().numpy())


def test_graph_replays_equal_launch_by_launch_iterations():
    """The solve loop replays one captured iteration as a HIP graph; with every
    launch timed it launches every kernel itself; with the analysis timed it
    launches the analysis and replays the rest.  All give the same bits, for
    one map and for a batch, and the graph path gives them again on a second
    solve (thousands of replays, host synchronisations in between)."""
    dev = device()
    nside, nmaps = 8, 3
    ps, T, ds = _members(nside, nmaps, first=40)
    lmax = ps[0].lmax
    args = (_stack([p.cl for p in ps], dev), _stack(ds, dev), _stack([p.ninv for p in ps], dev))
    for plan, sel in ((_plan(nside, lmax, nmaps), slice(None)), (_plan(nside, lmax, 1), 0)):
        a_in = tuple(x[sel].contiguous() for x in args)
        plan.profile(True)
        a_e, s_e, st_e = plan.solve(*a_in, eps_final=1e-8)
        plan.profile_read()
        plan.profile(False)
        a_g, s_g, st_g = plan.solve(*a_in, eps_final=1e-8)
        a_g2, s_g2, _ = plan.solve(*a_in, eps_final=1e-8)
        plan.profile(2)   # analysis timed between events, the rest replayed
        a_s, s_s, _ = plan.solve(*a_in, eps_final=1e-8)
        prof = plan.profile_read()
        plan.profile(False)
        assert prof["legendre_analysis"][0] > 0 and prof["legendre_synthesis"][0] == 0
        for x, y in ((a_e, a_g), (s_e, s_g), (a_g, a_g2), (s_g, s_g2), (a_e, a_s), (s_e, s_s)):
            np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
        st_e = st_e if isinstance(st_e, list) else [st_e]
        st_g = st_g if isinstance(st_g, list) else [st_g]
        assert [s.iters_per_level for s in st_e] == [s.iters_per_level for s in st_g]


def test_plans_solving_at_once_from_threads():
    """Plans of different Nside solving at the same time, each on its own
    stream from its own host thread (the batched workload's groups), give the
    bits each gives alone."""
    import threading
    import torch
    dev = device()
    jobs = []
    for nside, nmaps, first in ((4, 3, 50), (8, 2, 60)):
        ps, T, ds = _members(nside, nmaps, first=first)
        plan = _plan(nside, ps[0].lmax, nmaps)
        args = (_stack([p.cl for p in ps], dev), _stack(ds, dev), _stack([p.ninv for p in ps], dev))
        alone = plan.solve(*args, eps_final=1e-8)
        jobs.append((plan, args, alone))
    torch.cuda.synchronize()
    out = [None] * len(jobs)
    streams = [torch.cuda.Stream(device=dev) for _ in jobs]

    def run(i):
        plan, args, _ = jobs[i]
        with torch.cuda.stream(streams[i]):
            out[i] = plan.solve(*args, eps_final=1e-8)
        streams[i].synchronize()

    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for (plan, args, alone), got in zip(jobs, out):
        np.testing.assert_array_equal(got[0].cpu().numpy(), alone[0].cpu().numpy())
        np.testing.assert_array_equal(got[1].cpu().numpy(), alone[1].cpu().numpy())


# --------------------------------------------------------------------------
# several plans (groups of different Nside) solved from one graph
# --------------------------------------------------------------------------
def _group(nside, n, first, prec=0):
    from paper_1702_08852_amd import Plan
    dev = device()
    ps, T, ds = _members(nside, n, first)
    plan = Plan(nside, ps[0].lmax, nmaps=n, device=dev, precision=prec)
    st = lambda xs: torch_tensor(np.stack(xs) if n > 1 else xs[0], dev)
    return plan, (st([p.cl for p in ps]), st(ds), st([p.ninv for p in ps]))


@pytest.mark.parametrize("precs", [(0, 0, 0), (1, 0, 2)])
def test_solve_plans_equals_each_plans_own_solve(precs):
    """Three groups of the batched workload's recipe at Nside 4, 8 and 16 (in
    FP64, or one group per precision form) iterate from one graph; every map
    comes out bit for bit as its plan's own dmwf_solve gives it, with the same
    counts per level, and the replayed form of the call too."""
    from paper_1702_08852_amd import solve_plans
    groups = [_group(4, 2, 0, precs[0]), _group(8, 3, 2, precs[1]), _group(16, 1, 5, precs[2])]
    plans = [g[0] for g in groups]
    cls, ds, ws = ([g[1][i] for g in groups] for i in range(3))
    together = solve_plans(plans, cls, ds, ws, eps_final=1e-8, want_residual=True)
    for (plan, args), (a, m, sts) in zip(groups, together):
        a1, m1, st1 = plan.solve(*args, eps_final=1e-8, want_residual=True)
        np.testing.assert_array_equal(a.cpu().numpy(), a1.cpu().numpy())
        np.testing.assert_array_equal(m.cpu().numpy(), m1.cpu().numpy())
        sts = sts if isinstance(sts, list) else [sts]
        st1 = st1 if isinstance(st1, list) else [st1]
        for s_, t_ in zip(sts, st1):
            assert s_.status == 0 and s_.iters_per_level == t_.iters_per_level
            assert s_.iters_reduced == t_.iters_reduced and s_.wf_residual == t_.wf_residual
    # replayed: a mu0 small enough that every map's schedule is one coarse
    # level and the last (beta xi_0 <= alpha), so the counts fit every map
    mu0 = 0.5 * min(float(1.0 / w.max()) * 0.25 / (0.75 * 12 * pl.nside ** 2 / (4 * np.pi))
                    for pl, w in zip(plans, ws))
    ref = [plan.solve(*args, eps_final=1e-8, eps_coarse=1e-4, mu0=mu0, replay=[3, 4])
           for plan, args in groups]
    rep = solve_plans(plans, cls, ds, ws, eps_final=1e-8, mu0=mu0, replay=[3, 4])
    for (a1, m1, _), (a, m, _) in zip(ref, rep):
        np.testing.assert_array_equal(a.cpu().numpy(), a1.cpu().numpy())
        np.testing.assert_array_equal(m.cpu().numpy(), m1.cpu().numpy())


def test_solve_plans_with_analysis_timing_and_argument_errors():
    """Kernel timing of the analysis on one plan (launched between its events,
    the rest from the graph) changes no bits; a plan given twice is refused
    before any work."""
    from paper_1702_08852_amd import DmwfError, solve_plans
    from paper_1702_08852_amd import dmwf as b
    g1, g2 = _group(8, 2, 0), _group(16, 1, 3)
    base = solve_plans([g1[0], g2[0]], [g1[1][0], g2[1][0]], [g1[1][1], g2[1][1]],
                       [g1[1][2], g2[1][2]], eps_final=1e-8)
    g2[0].profile(2)
    timed = solve_plans([g1[0], g2[0]], [g1[1][0], g2[1][0]], [g1[1][1], g2[1][1]],
                        [g1[1][2], g2[1][2]], eps_final=1e-8)
    prof = g2[0].profile_read()
    g2[0].profile(False)
    assert prof["legendre_analysis"][0] > 0
    for (a, m, _), (a1, m1, _) in zip(base, timed):
        np.testing.assert_array_equal(a.cpu().numpy(), a1.cpu().numpy())
        np.testing.assert_array_equal(m.cpu().numpy(), m1.cpu().numpy())
    with pytest.raises(DmwfError) as e:
        solve_plans([g1[0], g1[0]], [g1[1][0]] * 2, [g1[1][1]] * 2, [g1[1][2]] * 2)
    assert e.value.status == b.ERR_INVALID_ARG
