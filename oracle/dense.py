"""The Wiener filter equation solved directly (small Nside only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Wiener filter equation of the paper's Section 1, (S^-1 + N^-1) s_WF = N^-1 d,
for the data model d = s + n.  On the sphere the signal is s = Y a with S = diag(C_l) in the a_lm
basis, so with W = N^-1 (zero on masked pixels) the same equation reads, in
harmonic space,

    (C^-1 + Y^H W Y) a_WF = Y^H W d,      s_WF = Y a_WF,

over the modes with C_l > 0 (a_lm = 0 elsewhere).  It is written here over the
real parameters of a real field (Re a_l0; Re and Im a_lm for m > 0), where the
design matrix has columns lambda_l0, 2 lambda_lm cos(m phi) and
-2 lambda_lm sin(m phi), and the prior precision is 1/C_l for m = 0 and 2/C_l
for each of Re, Im when m > 0 (E|a_lm|^2 = C_l).  The system is solved with a
dense Cholesky factorisation.

The fixed point of one cooling level of the dual messenger is the same
equation with the truncated spectrum S_bar = max(C - mu, 0) and the noise
N + (xi - alpha), i.e. weights w / (1 + (xi - alpha) w): minimise the hybrid
chi^2 (paper eq. chi2_hybrid_messenger) over t, whose marginal covariance for
d - s is N_bar + xi = N + (xi - alpha).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import lambda_lm, n_alm, rings


def real_design(nside: int, lmax: int, active_l: np.ndarray):
    """Real design matrix [npix, nparam] and the (slot, part, m) of every column.

    active_l[l] selects which multipoles enter.  part 0 = Re, 1 = Im.
    """
    z, st, nph, p0, start = rings(nside)
    npix = 12 * nside * nside
    cols = []
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            if not active_l[l]:
                continue
            slot = m * (2 * lmax + 1 - m) // 2 + l
            cols.append((slot, 0, m, l))
            if m > 0:
                cols.append((slot, 1, m, l))
    Yr = np.zeros((npix, len(cols)))
    col_of = {}
    for j, (slot, part, m, l) in enumerate(cols):
        col_of[(slot, part)] = j
    for k in range(len(z)):
        s, n = start[k], nph[k]
        phi = p0[k] + 2.0 * math.pi * np.arange(n) / n
        for m in range(lmax + 1):
            lam = lambda_lm(m, z[k], st[k], lmax)
            cm, sm = np.cos(m * phi), np.sin(m * phi)
            for l in range(m, lmax + 1):
                if not active_l[l]:
                    continue
                slot = m * (2 * lmax + 1 - m) // 2 + l
                if m == 0:
                    Yr[s:s + n, col_of[(slot, 0)]] = lam[l - m]
                else:
                    Yr[s:s + n, col_of[(slot, 0)]] = 2.0 * lam[l - m] * cm
                    Yr[s:s + n, col_of[(slot, 1)]] = -2.0 * lam[l - m] * sm
    return Yr, cols


def wiener_dense(nside: int, lmax: int, cl: np.ndarray, w: np.ndarray, d: np.ndarray,
                 design=None) -> np.ndarray:
    """a_WF [n_alm, 2] solving (C^-1 + Y^H W Y) a = Y^H W d over modes with C_l > 0."""
    cl = np.asarray(cl, dtype=np.float64)
    active = cl > 0.0
    Yr, cols = design if design is not None else real_design(nside, lmax, active)
    prec = np.array([(1.0 if m == 0 else 2.0) / cl[l] for (_, _, m, l) in cols])
    A = Yr.T @ (w[:, None] * Yr)
    A[np.diag_indices_from(A)] += prec
    b = Yr.T @ (w * d)
    x = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    out = np.zeros((n_alm(lmax), 2))
    for j, (slot, part, _, _) in enumerate(cols):
        out[slot, part] = x[j]
    return out


def level_fixed_point(nside: int, lmax: int, cl: np.ndarray, w: np.ndarray, d: np.ndarray,
                      xi: float, alpha: float, sigma: float) -> np.ndarray:
    """Fixed point of the cooling level xi: the filter with S_bar and N + (xi - alpha)."""
    mu = (xi - alpha) / sigma
    sbar = np.where(cl - mu > 0.0, cl - mu, 0.0)
    w_xi = w / (1.0 + (xi - alpha) * w)
    return wiener_dense(nside, lmax, sbar, w_xi, d)
