"""CPU reference of the warm-start network (features, forward, loss, gradient,
Adam step) in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The GPU network's
kernels are checked against these functions; these functions are pinned by
finite differences of the loss, the closed form of Adam's first step and
index properties of the feature window (tests/test_oracle_nn.py).

The network (a component outside the paper, whose solver starts from zero):
per mode (l, m), features -> 128 -> 128 -> 2 with ReLU after the first two
layers; parameters flat as W1 [24][128], b1, W2 [128][128], b2, W3 [128][2],
b3 (y = x W + b).  Loss: mean over the rows of |y - t|^2.
"""
from __future__ import annotations

import math

import numpy as np

F, H, O = 24, 128, 2
SHAPES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, O)),
          ("b3", (O,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
WIN = 4


def unflatten(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def slot_lm(lmax):
    """(l, m) of every m-major a_lm slot."""
    ls, ms = [], []
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            ls.append(l)
            ms.append(m)
    return np.array(ls), np.array(ms)


def features(dlm, cl, lmax, noise_w, fsky, slots):
    """Feature rows of the listed slots (see the network's definition)."""
    dlm = np.asarray(dlm, dtype=np.float64).reshape(-1, 2)
    ls, ms = slot_lm(lmax)
    x = np.zeros((len(slots), F))
    for r, s in enumerate(slots):
        l, m = int(ls[s]), int(ms[s])
        c = float(cl[l])
        if l < 2 or c <= 0.0:
            continue
        scale = 1.0 / math.sqrt(c + noise_w)
        base = m * (2 * lmax + 1 - m) // 2
        for k in range(-WIN, WIN + 1):
            lk = l + k
            if m <= lk <= lmax:
                x[r, 2 * (k + WIN)] = dlm[base + lk, 0] * scale
                x[r, 2 * (k + WIN) + 1] = 0.0 if m == 0 else dlm[base + lk, 1] * scale
        x[r, 18] = c / (c + noise_w)
        x[r, 19] = m / (l + 1.0)
        x[r, 20] = fsky
        x[r, 21] = math.log10(noise_w / c) / 10.0
    return x


def targets(alm, cl, lmax, slots):
    """Whitened Wiener filter coefficients a_lm / sqrt(C_l) of the listed slots."""
    alm = np.asarray(alm, dtype=np.float64).reshape(-1, 2)
    ls, ms = slot_lm(lmax)
    t = np.zeros((len(slots), O))
    for r, s in enumerate(slots):
        l, m = int(ls[s]), int(ms[s])
        if l < 2 or cl[l] <= 0.0:
            continue
        t[r, 0] = alm[s, 0] / math.sqrt(cl[l])
        t[r, 1] = 0.0 if m == 0 else alm[s, 1] / math.sqrt(cl[l])
    return t


def forward(p, x):
    """(y, cache) for rows x."""
    P = unflatten(p)
    z1 = x @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"] + P["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t):
    y, _ = forward(p, x)
    return float(np.sum((y - t) ** 2) / x.shape[0])


def loss_and_grad(p, x, t):
    """Loss and its gradient with respect to the flat parameters (backpropagation)."""
    P = unflatten(p)
    y, (x, z1, h1, z2, h2) = forward(p, x)
    n = x.shape[0]
    gy = 2.0 * (y - t) / n
    g = {"W3": h2.T @ gy, "b3": gy.sum(axis=0)}
    gz2 = (gy @ P["W3"].T) * (z2 > 0.0)
    g["W2"] = h1.T @ gz2
    g["b2"] = gz2.sum(axis=0)
    gz1 = (gz2 @ P["W2"].T) * (z1 > 0.0)
    g["W1"] = x.T @ gz1
    g["b1"] = gz1.sum(axis=0)
    return float(np.sum((y - t) ** 2) / n), flatten(g)


def adam_step(p, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) at step number `step` (1-based)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2
