"""GPU path against the oracle at the workload sizes.

Full transforms up to Nside 512; at the paper-scale Nside 1024 / lmax 2048
(the benchmark's launch configuration) the oracle evaluates sampled rings and
sampled m one by one, one full iteration through the C ABI is checked
against an oracle iteration, and solves replayed across level switches
(Nside 1024 and 256) are checked in a, s and the FP64 residual.  The batched
workload's Nside 512 group is checked the same way in its autotuned launch
configuration.
"""
import math

import numpy as np
import pytest

import dmwf_inputs as inp
import oracle
from oracle import dm
from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu


def _plan(nside, lmax):
    from paper_1702_08852_amd import Plan
    return Plan(nside, lmax, device=device())


@pytest.mark.parametrize("nside,lmax", [(128, 256), (256, 512), (512, 1024)])
def test_transforms_full(nside, lmax):
    dev = device()
    a = inp.random_alm(lmax, 7 + nside)
    plan = _plan(nside, lmax)
    got = plan.alm2map(to_dev(a, dev)).cpu().numpy()
    assert rel(got, oracle.alm2map(a, nside, lmax)) < 1e-12
    mp = inp.random_map(nside, 9 + nside)
    got = plan.adjoint(to_dev(mp, dev)).cpu().numpy()
    assert rel(got, oracle.adjoint(mp, nside, lmax)) < 1e-12


RINGS_1024 = [1, 2, 3, 4, 100, 511, 512, 1023, 1024, 1025, 1500, 2047, 2048, 2049, 3000, 3071,
              3072, 3073, 4000, 4093, 4094, 4095]
MS_2048 = [0, 1, 2, 3, 50, 511, 512, 1000, 1023, 1024, 1500, 2000, 2046, 2047, 2048]


def test_alm2map_nside1024_sampled_rings():
    dev = device()
    nside, lmax = 1024, 2048
    a = inp.random_alm(lmax, 1024)
    got = _plan(nside, lmax).alm2map(to_dev(a, dev)).cpu().numpy()
    z, st, nph, p0, start = oracle.rings(nside)
    ref = oracle.alm2map_rings(a, nside, lmax, RINGS_1024)
    mine = np.concatenate([got[start[r - 1]:start[r - 1] + nph[r - 1]] for r in RINGS_1024])
    assert rel(mine, ref) < 1e-12
    o = 0
    for r in RINGS_1024:  # every sampled ring on its own
        n = nph[r - 1]
        assert rel(mine[o:o + n], ref[o:o + n]) < 1e-11, r
        o += n


def test_adjoint_nside1024_sampled_m():
    dev = device()
    nside, lmax = 1024, 2048
    mp = inp.random_map(nside, 1025)
    got = _plan(nside, lmax).adjoint(to_dev(mp, dev)).cpu().numpy()
    ref = oracle.adjoint_m(mp, nside, lmax, MS_2048)
    for m, v in ref.items():
        k0 = oracle.alm_index(m, m, lmax)
        assert rel(got[k0:k0 + lmax - m + 1], v) < 1e-12, m


def _problem(name, nside):
    p = inp.make_problem(name, nside=nside)
    T = oracle.SphereTransforms(nside, p.lmax)
    d = p.data_map(T.synth(p.alm_true))
    return p, T, d, p.ninv


@pytest.mark.parametrize("level", [0, 20, -1])
def test_dm_iterate_nside256_cfg2(level):
    """Configuration 2 recipe (Nside 256, lmax 512): three iterations on one level."""
    import torch
    dev = device()
    nside = 256
    p, T, d, w = _problem("cfg2", nside)
    alpha = dm.alpha_of(w)
    sigma = 1.0 / T.omega
    xi = dm.level_schedule(alpha, sigma, p.cl, 0.75)[level]
    mu, f, li = dm.level_params(xi, alpha, sigma, p.cl)
    c = dm.pixel_coeff(xi, alpha, w)
    plan = _plan(nside, p.lmax)
    cl_t, d_t, w_t = to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev)
    a_t = torch.zeros((oracle.n_alm(p.lmax), 2), dtype=torch.float64, device=dev)
    s_t = torch.zeros(12 * nside * nside, dtype=torch.float64, device=dev)
    c2 = torch.zeros(2, dtype=torch.float64, device=dev)
    a = np.zeros((oracle.n_alm(p.lmax), 2))
    r = np.where(w > 0, d, 0.0)
    s_prev = np.zeros_like(d)
    for it in range(3):
        plan.dm_iterate(xi, alpha, cl_t, d_t, w_t, a_t, s_t, c2, first=(it == 0))
        a, s, r, num, den = dm.iterate(T, a, r, f[T.ell()], c, d, s_prev)
        s_prev = s
        assert rel(a_t.cpu().numpy(), a) < 1e-11
        assert rel(s_t.cpu().numpy(), s) < 1e-11
        cc = c2.cpu().numpy()
        assert cc[1] == pytest.approx(den, rel=1e-11)
        assert cc[0] == pytest.approx(num, rel=1e-8, abs=1e-13 * den)


def test_dm_iterate_nside1024_cfg3_first_iteration():
    """Configuration 3 recipe at full size: the first iteration at the final level xi = alpha."""
    import torch
    dev = device()
    nside = 1024
    p, T, d, w = _problem("cfg3", nside)
    assert abs(p.meta["masked_fraction"] - 0.20) < 0.005
    alpha = dm.alpha_of(w)
    sigma = 1.0 / T.omega
    xi = alpha
    mu, f, li = dm.level_params(xi, alpha, sigma, p.cl)
    plan = _plan(nside, p.lmax)
    cl_t, d_t, w_t = to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev)
    a_t = torch.zeros((oracle.n_alm(p.lmax), 2), dtype=torch.float64, device=dev)
    s_t = torch.zeros(12 * nside * nside, dtype=torch.float64, device=dev)
    c2 = torch.zeros(2, dtype=torch.float64, device=dev)
    plan.dm_iterate(xi, alpha, cl_t, d_t, w_t, a_t, s_t, c2, first=True)
    a_gpu = a_t.cpu().numpy()
    s_gpu = s_t.cpu().numpy()
    # oracle: a_1 = f (Omega Y^H d[w>0]) in full, s_1 = Y a_1 on sampled rings
    r0 = np.where(w > 0, d, 0.0)
    a1 = f[T.ell()][:, None] * (T.omega * T.adjoint(r0))
    assert rel(a_gpu, a1) < 1e-11
    z, st, nph, p0, start = oracle.rings(nside)
    ref = oracle.alm2map_rings(a1, nside, p.lmax, RINGS_1024)
    mine = np.concatenate([s_gpu[start[r - 1]:start[r - 1] + nph[r - 1]] for r in RINGS_1024])
    assert rel(mine, ref) < 1e-11
    cc = c2.cpu().numpy()
    assert math.isfinite(cc[0]) and cc[0] == pytest.approx(cc[1], rel=1e-12)  # s_prev = 0


def test_batched_nside512_group_sampled():
    """The batched workload's Nside 512 group (16 maps of its own recipe) in the
    autotuned launch configuration the benchmark times: batched transforms on
    sampled rings and m of first, middle and last maps, and one full-band
    iteration of the batched solve against the oracle for two maps."""
    import torch
    from paper_1702_08852_amd import Plan
    dev = device()
    nside, lmax = 512, 1024
    idx = inp.batch_members(nside)
    nm = len(idx)
    plan = Plan(nside, lmax, nmaps=nm, device=dev)
    plan.autotune()
    a = np.stack([inp.random_alm(lmax, 900 + k) for k in range(nm)])
    got = plan.alm2map(torch.tensor(a, device=dev)).cpu().numpy()
    z, st, nph, p0, start = oracle.rings(nside)
    rings = [1, 2, 255, 256, 511, 512, 1000, 1023, 1024, 1025, 2000, 2046, 2047]
    for k in (0, 7, nm - 1):
        ref = oracle.alm2map_rings(a[k], nside, lmax, rings)
        mine = np.concatenate([got[k, start[r - 1]:start[r - 1] + nph[r - 1]] for r in rings])
        assert rel(mine, ref) < 1e-12, k
    mp = np.stack([inp.random_map(nside, 950 + k) for k in range(nm)])
    got = plan.adjoint(torch.tensor(mp, device=dev)).cpu().numpy()
    ms = [0, 1, 255, 256, 511, 512, 1000, 1023, 1024]
    for k in (0, nm - 1):
        ref = oracle.adjoint_m(mp[k], nside, lmax, ms)
        for m, v in ref.items():
            k0 = oracle.alm_index(m, m, lmax)
            assert rel(got[k, k0:k0 + lmax - m + 1], v) < 1e-12, (k, m)
    # one full-band iteration at xi = alpha from a = 0, every map at once
    probs = [inp.make_problem("cfg4", nside=nside, index=i) for i in idx]
    T = oracle.SphereTransforms(nside, lmax)
    ds = [q.data_map(T.synth(q.alm_true)) for q in probs[:2]]
    d = np.stack(ds + [probs[k].sigma * probs[k].white * ~probs[k].mask for k in range(2, nm)])
    w = np.stack([q.ninv for q in probs])
    cl = np.stack([q.cl for q in probs])
    a0 = torch.zeros((nm, oracle.n_alm(lmax), 2), dtype=torch.float64, device=dev)
    alm, smap, sts = plan.solve(torch.tensor(cl, device=dev), torch.tensor(d, device=dev),
                                torch.tensor(w, device=dev), start_final=True, alm=a0,
                                replay=[1])
    res = plan.wf_residual(torch.tensor(cl, device=dev), torch.tensor(d, device=dev),
                           torch.tensor(w, device=dev), alm)
    alm, smap = alm.cpu().numpy(), smap.cpu().numpy()
    for k in range(2):
        ref = dm.solve(T, d[k], w[k], cl[k], start_final=True, alm0=np.zeros_like(alm[k]),
                       replay=[1])
        assert sts[k].n_iter == 1 and ref.n_iter == 1
        assert rel(alm[k], ref.alm) < 1e-11
        assert rel(smap[k], ref.map) < 1e-11
        # the batched residual of map k against the oracle's
        assert res[k] == pytest.approx(dm.wf_residual(T, ref.alm, d[k], w[k], cl[k]), rel=1e-8)


def _solve_and_replay(nside, name, mu0, replay_gpu, replay_oracle, cap, ring_list):
    """dmwf_solve through the C ABI with replayed per-level counts and an
    iteration cap, against the oracle replaying the same counts; returns the
    GPU stats and the oracle result after comparing a and s."""
    dev = device()
    p, T, d, w = _problem(name, nside)
    plan = _plan(nside, p.lmax)
    alm, smap, st = plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev), mu0=mu0,
                               eps_final=1e-6, eps_coarse=1e-4, replay=replay_gpu, max_iter=cap)
    alm, smap = alm.cpu().numpy(), smap.cpu().numpy()
    ref = dm.solve(T, d, w, p.cl, mu0=mu0, eps_final=1e-6, eps_coarse=1e-4, replay=replay_oracle,
                   max_iter=cap)
    assert st.n_iter == ref.n_iter == cap
    nl = len(st.iters_per_level)
    assert st.iters_per_level == list(ref.iters_per_level)
    assert st.lmax_per_level == ref.ell_iters[:nl]
    np.testing.assert_allclose(st.xi_per_level, ref.xis[:nl], rtol=1e-15)
    assert rel(alm, ref.alm) < 1e-10
    assert rel(smap, ref.map) < 1e-10
    z, st_, nph, p0, start = oracle.rings(nside)
    for r in ring_list:  # every sampled ring on its own
        sl = slice(start[r - 1], start[r - 1] + nph[r - 1])
        assert rel(smap[sl], ref.map[sl]) < 1e-10, r
    # the FP64 residual of the Wiener filter system at the solve's end point
    # (its own ring-stage modes: synthesis with the weighted residual, then
    # the weighted-data analysis) against the oracle's at the oracle's
    got = plan.wf_residual(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev), to_dev(alm, dev))
    want = dm.wf_residual(T, ref.alm, d, w, p.cl)
    print(f"nside {nside}: wf_residual {got:.6e} oracle {want:.6e}")
    assert got == pytest.approx(want, rel=1e-8)
    return st, ref, p


def test_solve_nside1024_cfg3_across_level_switches():
    """Configuration 3 at full size (Nside 1024, lmax 2048) through dmwf_solve:
    level 0 starts mid-band (mu0 = C_500, l_iter near 500), one iteration on
    each of levels 0 and 1 and two on level 2, stopped by the iteration cap.
    This runs the device level control across two level switches (k_control,
    the per-level m bounds of every ring pair, the unfold of G to the next
    level's l_iter) with every ring-length class, and ends on iterations whose
    previous s is not zero."""
    from paper_1702_08852_amd import dmwf as b
    nside = 1024
    p0 = inp.make_problem("cfg3", nside=nside)
    mu0 = float(p0.cl[500])
    nlev = len(dm.level_schedule(dm.alpha_of(p0.ninv), 12 * nside * nside / (4 * math.pi),
                                 p0.cl, 0.75, mu0))
    st, ref, p = _solve_and_replay(nside, "cfg3", mu0, [1, 1, 5] + [1] * (nlev - 3),
                                   [1, 1, 1000] + [1] * (nlev - 3), 4, RINGS_1024)
    assert st.status == b.ERR_NOT_CONVERGED
    assert st.iters_per_level == [1, 1, 2]
    ells = st.lmax_per_level
    assert 400 <= ells[0] < ells[1] < ells[2] < p.lmax  # the band grows with every switch


def test_solve_nside256_cfg2_every_level_replayed():
    """Configuration 2 (Nside 256, lmax 512) through dmwf_solve over its whole
    cooling schedule (every level, two iterations each, three on the last):
    the device level control at every switch up to xi = alpha against the
    oracle replaying the same counts."""
    nside = 256
    p0 = inp.make_problem("cfg2", nside=nside)
    nlev = len(dm.level_schedule(dm.alpha_of(p0.ninv), 12 * nside * nside / (4 * math.pi),
                                 p0.cl, 0.75))
    rep = [2] * (nlev - 1) + [3]
    st, ref, p = _solve_and_replay(nside, "cfg2", -1.0, rep, rep, sum(rep),
                                   [1, 2, 100, 255, 256, 257, 511, 512, 513, 700, 1022, 1023])
    assert st.status == 0 and len(st.iters_per_level) == nlev >= 5
    assert st.lmax_per_level[-1] == p.lmax
