"""The warm-start network's HIP kernels against the CPU reference
(oracle/nn.py): features, forward pass, gradient of the batch loss, Adam
steps, the warm start of a whole map, and solves entering from a warm start.

FP32 bars: features 1e-6 (inputs rounded to FP32); forward 1e-5 and
gradients 1e-4 relative L2 per parameter block (FP32 products summed over
128 terms per layer and over the batch for the weight gradients).
"""
import numpy as np
import pytest

import dmwf_inputs as inp
import oracle
from oracle import dm, nn
from gpu_util import device, rel, to_dev

pytestmark = pytest.mark.gpu


def _f32(a, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)


def _blocks(a):
    out, o = {}, 0
    for name, shp in nn.SHAPES:
        n = int(np.prod(shp))
        out[name] = a[o:o + n]
        o += n
    return out


def _net(dev, seed=1, max_batch=4096):
    from paper_1702_08852_amd import Net
    net = Net(max_batch=max_batch, device=dev)
    p = inp.nn_init_params(seed)
    rng = np.random.default_rng(seed)
    p = (p + 0.05 * rng.standard_normal(p.size)).astype(np.float32)
    net.set_params(_f32(p, dev))
    return net, p.astype(np.float64)


@pytest.mark.parametrize("lmax", [9, 40])
def test_features_match_reference(lmax):
    import torch
    from paper_1702_08852_amd import nn_features
    dev = device()
    nalm = (lmax + 1) * (lmax + 2) // 2
    rng = np.random.default_rng(lmax)
    dlm = rng.standard_normal((nalm, 2))
    alm = rng.standard_normal((nalm, 2))
    cl = inp.cl_damped(lmax, lcut=lmax / 2.0)
    x, t = nn_features(lmax, to_dev(dlm, dev), to_dev(cl, dev), 0.02, 0.8, n=nalm,
                       target=to_dev(alm, dev))
    slots = list(range(nalm))
    assert rel(x.cpu().numpy(), nn.features(dlm, cl, lmax, 0.02, 0.8, slots)) < 1e-6
    assert rel(t.cpu().numpy(), nn.targets(alm, cl, lmax, slots)) < 1e-6
    pick = rng.permutation(nalm)[:nalm // 3].astype(np.int32)
    xs, _ = nn_features(lmax, to_dev(dlm, dev), to_dev(cl, dev), 0.02, 0.8,
                        slots=torch.tensor(pick, device=dev))
    assert rel(xs.cpu().numpy(), nn.features(dlm, cl, lmax, 0.02, 0.8, list(pick))) < 1e-6


@pytest.mark.parametrize("n", [1, 63, 1000, 4096])
def test_forward_and_gradient_match_reference(n):
    """Batches from one row to max_batch, ragged against the 64-row tiles."""
    dev = device()
    net, p = _net(dev)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, nn.F)).astype(np.float32)
    t = rng.standard_normal((n, nn.O)).astype(np.float32)
    y = net.forward(_f32(x, dev)).cpu().numpy()
    yr, _ = nn.forward(p, x.astype(np.float64))
    assert rel(y, yr) < 1e-5
    g, loss = net.gradient(_f32(x, dev), _f32(t, dev))
    Lr, gr = nn.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(Lr, rel=1e-5)
    gb, rb = _blocks(g.cpu().numpy()), _blocks(gr)
    for name in gb:
        assert rel(gb[name], rb[name]) < 1e-4, name


def test_adam_steps_match_reference_and_learn():
    """Three Adam steps on one batch follow the reference step by step; forty
    steps on a linear target cut the loss."""
    import torch
    dev = device()
    net, p = _net(dev, seed=2)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((512, nn.F)).astype(np.float32)
    t = (x[:, :2] * 0.5 + 0.1).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    m1 = np.zeros_like(p)
    m2 = np.zeros_like(p)
    q = p.copy()
    for step in range(1, 4):
        net.train_step(_f32(x, dev), _f32(t, dev), 1e-3, loss)
        Lr, g = nn.loss_and_grad(q, x.astype(np.float64), t.astype(np.float64))
        q, m1, m2 = nn.adam_step(q, g, m1, m2, step, 1e-3)
        assert float(loss.cpu()[0]) == pytest.approx(Lr, rel=1e-5)
        got = _blocks(net.params().cpu().numpy())
        for name, v in _blocks(q).items():
            assert rel(got[name], v) < 1e-5, (step, name)
    first = None
    for _ in range(40):
        net.train_step(_f32(x, dev), _f32(t, dev), 1e-3, loss)
        first = float(loss.cpu()[0]) if first is None else first
    assert float(loss.cpu()[0]) < 0.5 * first


def test_warm_start_of_a_map_matches_reference():
    """The network's a_lm estimate of a map (features of every slot, forward
    in max_batch pieces, un-whitening) equals the reference network applied to
    the reference features."""
    from paper_1702_08852_amd import Plan, noise_stats
    dev = device()
    nside = 16
    p = inp.make_problem("cfg5", nside=nside, index=3)
    T = oracle.SphereTransforms(nside, p.lmax)
    d = p.data_map(T.synth(p.alm_true))
    net, prm = _net(dev, seed=4, max_batch=200)  # several pieces
    plan = Plan(nside, p.lmax, device=dev)
    dlm = plan.adjoint(to_dev(d, dev), scale_by_pixel_area=True)
    nw, fsky = noise_stats(to_dev(p.ninv, dev))
    w = p.ninv
    assert nw == pytest.approx(T.omega / w[w > 0].mean(), rel=1e-12)
    assert fsky == pytest.approx((w > 0).mean(), rel=1e-12)
    a0 = net.warm_start(p.lmax, dlm, to_dev(p.cl, dev), nw, fsky).cpu().numpy()
    nalm = oracle.n_alm(p.lmax)
    xr = nn.features(dlm.cpu().numpy(), p.cl, p.lmax, nw, fsky, list(range(nalm)))
    yr, _ = nn.forward(prm, xr)
    ls, ms = nn.slot_lm(p.lmax)
    want = yr * np.sqrt(p.cl[ls])[:, None]
    want[ls < 2] = 0.0
    want[ms == 0, 1] = 0.0
    assert rel(a0, want) < 1e-5


@pytest.mark.parametrize("final", [False, True])
def test_solve_from_a_warm_start_matches_oracle(final):
    """A solve entering from given a_lm (the whole cooling schedule, or the
    last level only) against the oracle started from the same a_lm, replaying
    its counts (FP64 parity bar)."""
    dev = device()
    nside = 8
    p = inp.make_problem("cfg1", nside=nside)
    T = oracle.SphereTransforms(nside, p.lmax)
    d = p.data_map(T.synth(p.alm_true))
    w = p.ninv
    a0 = 0.6 * p.alm_true
    a0[:p.lmax + 1, 1] = 0.0
    ref = dm.solve(T, d, w, p.cl, eps_final=1e-8, eps_coarse=1e-4, alm0=a0, start_final=final)
    from paper_1702_08852_amd import Plan
    plan = Plan(nside, p.lmax, device=dev)
    alm, smap, st = plan.solve(to_dev(p.cl, dev), to_dev(d, dev), to_dev(w, dev), eps_final=1e-8,
                               eps_coarse=1e-4, alm=to_dev(a0, dev), start_final=final,
                               warm_start=not final, replay=ref.iters_per_level)
    assert st.iters_per_level == list(ref.iters_per_level)
    assert rel(alm.cpu().numpy(), ref.alm) < 1e-10
    assert rel(smap.cpu().numpy(), ref.map) < 1e-10
