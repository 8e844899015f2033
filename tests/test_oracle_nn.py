"""Pins of the CPU reference of the warm-start network (oracle/nn.py).

The gradient is checked against central finite differences of the loss, the
Adam step against its closed form at the first step, the forward pass
against a hand-built network in its linear region, and the feature window
against single-coefficient inputs whose images are known by construction.
"""
import math

import numpy as np
import pytest

import dmwf_inputs as inp
from oracle import nn


def _params(seed=1):
    rng = np.random.default_rng(seed)
    p = inp.nn_init_params(seed).astype(np.float64)
    return p + 0.05 * rng.standard_normal(p.size)  # nonzero biases: no unit sits at a kink


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    p = _params()
    x = rng.standard_normal((17, nn.F))
    t = rng.standard_normal((17, nn.O))
    L, g = nn.loss_and_grad(p, x, t)
    assert L == pytest.approx(nn.loss(p, x, t), rel=1e-14)
    # a sample of every block: first and last entries and random ones
    idx, o = [], 0
    for name, shp in nn.SHAPES:
        n = int(np.prod(shp))
        idx += [o, o + n - 1] + list(o + rng.integers(0, n, 6))
        o += n
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (nn.loss(p + e, x, t) - nn.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (abs(fd) + 1e-3 * np.abs(g).max()), i


def test_adam_first_step_is_lr_times_sign():
    """At step 1 the bias-corrected moments are g and g^2, so each parameter
    moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    q, m1, m2 = nn.adam_step(p, g, z, z, 1, 1e-3)
    np.testing.assert_allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(m2, 0.001 * g * g, rtol=1e-14)


def test_forward_in_the_linear_region():
    """With positive inputs, weights and biases every ReLU passes its input, so
    y = ((x W1 + b1) W2 + b2) W3 + b3."""
    rng = np.random.default_rng(3)
    P = {"W1": rng.uniform(0, 1, (nn.F, nn.H)), "b1": rng.uniform(0, 1, nn.H),
         "W2": rng.uniform(0, 1, (nn.H, nn.H)), "b2": rng.uniform(0, 1, nn.H),
         "W3": rng.standard_normal((nn.H, nn.O)), "b3": rng.standard_normal(nn.O)}
    x = rng.uniform(0, 1, (5, nn.F))
    want = ((x @ P["W1"] + P["b1"]) @ P["W2"] + P["b2"]) @ P["W3"] + P["b3"]
    y, _ = nn.forward(nn.flatten(P), x)
    np.testing.assert_allclose(y, want, rtol=1e-12)
    # and a unit driven negative is cut: b1 = -big switches layer 1 off
    P["b1"] = -1e6 * np.ones(nn.H)
    y, _ = nn.forward(nn.flatten(P), x)
    want = np.maximum(P["b2"], 0) @ P["W3"] + P["b3"]
    np.testing.assert_allclose(y, np.broadcast_to(want, y.shape), rtol=1e-12, atol=1e-12)


def test_feature_window_of_a_single_coefficient():
    """d_lm = 0 except (l0, m0) = (10, 3) = 1 + 2i: the rows (l, 3) with
    |l - 10| <= 4 see it at window position l0 - l + 4 (whitened by
    1 / sqrt(C_l + N_w) = 1/2), every other window entry is zero."""
    lmax, l0, m0 = 20, 10, 3
    nalm = (lmax + 1) * (lmax + 2) // 2
    dlm = np.zeros((nalm, 2))
    s0 = m0 * (2 * lmax + 1 - m0) // 2 + l0
    dlm[s0] = (1.0, 2.0)
    cl = np.full(lmax + 1, 2.0)
    x = nn.features(dlm, cl, lmax, 2.0, 0.7, list(range(nalm)))
    ls, ms = nn.slot_lm(lmax)
    for s in range(nalm):
        l, m = ls[s], ms[s]
        win = x[s, :18].reshape(9, 2)
        if l < 2:
            assert not x[s].any()
            continue
        if m == m0 and abs(l - l0) <= nn.WIN:
            k = l0 - l + nn.WIN
            np.testing.assert_allclose(win[k], (0.5, 1.0), rtol=1e-15)
            win = np.delete(win, k, axis=0)
        assert not win.any(), (l, m)
        assert x[s, 18] == pytest.approx(0.5)
        assert x[s, 19] == pytest.approx(m / (l + 1.0))
        assert x[s, 20] == 0.7 and x[s, 21] == 0.0


def test_features_edges_and_scaling():
    """m = 0 rows carry no imaginary part, window slots outside m..lmax are
    zero, the window scales with the data and the per-l features do not."""
    lmax = 12
    nalm = (lmax + 1) * (lmax + 2) // 2
    rng = np.random.default_rng(4)
    dlm = rng.standard_normal((nalm, 2))
    cl = inp.cl_damped(lmax, lcut=6.0)
    slots = list(range(nalm))
    x = nn.features(dlm, cl, lmax, 0.3, 0.5, slots)
    x3 = nn.features(3.0 * dlm, cl, lmax, 0.3, 0.5, slots)
    np.testing.assert_allclose(x3[:, :18], 3.0 * x[:, :18], rtol=1e-15)
    np.testing.assert_array_equal(x3[:, 18:], x[:, 18:])
    ls, ms = nn.slot_lm(lmax)
    for s in range(nalm):
        l, m = ls[s], ms[s]
        if l < 2:
            continue
        win = x[s, :18].reshape(9, 2)
        if m == 0:
            assert not win[:, 1].any()
        for k in range(-nn.WIN, nn.WIN + 1):
            if not (m <= l + k <= lmax):
                assert not win[k + nn.WIN].any()
        assert x[s, 21] == pytest.approx(math.log10(0.3 / cl[l]) / 10.0)
