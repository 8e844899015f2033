"""Dual messenger Wiener filter: the paper's Algorithm 2 (Section 2.2) in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method (paper Section 2.2, the hybrid form that fixes the zero eigenvalue
of S): the auxiliary field t has covariance xi = (alpha + mu) 1 with
alpha = min diag N (eq. for chi^2_xi); the signal prior is the truncated
spectrum S_bar = Theta(S - U) (Appendix B); xi is cooled geometrically,
xi <- beta xi, until xi = alpha where mu = 0 and the Wiener filter is reached.
Each cooling level repeats two diagonal solves,

    harmonic step   s_hat = [(S_bar^-1 + sigma xi^-1)^-1 sigma xi^-1] F(t)
    pixel step      t = (N_bar^-1 + xi^-1)^-1 (N_bar^-1 d + xi^-1 s)

until the Cauchy ratio ||s_i - s_{i-1}|| / ||s_i|| drops below epsilon.

Readings on the sphere:
  * F^-1 = Y (synthesis), F = Omega Y^H with Omega = 4 pi / Npix the pixel
    area, so sigma = 1/Omega; mu is in harmonic units, mu = (xi-alpha)/sigma,
    and the harmonic messenger variance is xi/sigma.
  * The pixel step uses N_bar = N - alpha (the hybrid minimisation equations),
    written with w = N^-1 so masked pixels (w = 0) are exact:
    t - s = c (d - s),  c = xi w / (1 + (xi - alpha) w).
  * The harmonic step is taken in residual form,
    a <- f (a + Omega Y^H (t - s)),  f_l = S_bar_l / (S_bar_l + xi/sigma),
    identical to f F(t) whenever F F^-1 = 1 (the paper's flat-sky FFT), and
    with the textbook Wiener filter as its fixed point on the HEALPix grid
    where Omega Y^H Y is only approximately the identity.
  * Theta(x) = x for x > 0 and 0 otherwise, so modes with C_l <= mu are zero.
  * Start: s = 0, t = d, i.e. the first residual is d on unmasked pixels.
  * Initial mu: mu0 = beta * max_l C_l unless given.  Levels: xi_0 = alpha +
    sigma mu0, xi_{k+1} = beta xi_k, and the first xi_{k+1} <= alpha is
    replaced by alpha, which is the last level.
  * Tolerance: eps_coarse on levels with xi > alpha, eps_final at xi = alpha.
  * Cauchy norm: unweighted L2 over all pixels; s_{i-1} carries over level
    boundaries; 0/0 counts as 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def alpha_of(w: np.ndarray) -> float:
    """alpha = min diag N over unmasked pixels = 1 / max w."""
    wmax = float(np.max(w)) if w.size else 0.0
    if not (wmax > 0.0):
        raise ValueError("every pixel is masked")
    return 1.0 / wmax


def level_schedule(alpha: float, sigma: float, cl: np.ndarray, beta: float,
                   mu0: float | None = None) -> list[float]:
    """The xi of every cooling level, ending with xi = alpha."""
    if mu0 is None or mu0 < 0:
        mu0 = beta * float(np.max(cl)) if cl.size else 0.0
    xi = alpha + sigma * mu0
    out = []
    while xi > alpha:
        out.append(xi)
        xi = beta * xi
    out.append(alpha)
    return out


def level_params(xi: float, alpha: float, sigma: float, cl: np.ndarray):
    """mu, the harmonic filter f_l and l_iter (largest l with S_bar_l > 0, or -1)."""
    mu = (xi - alpha) / sigma
    sbar = cl - mu
    sbar = np.where(sbar > 0.0, sbar, 0.0)
    f = sbar / (sbar + xi / sigma)
    act = np.nonzero(sbar > 0.0)[0]
    ell_iter = int(act[-1]) if act.size else -1
    return mu, f, ell_iter


def pixel_coeff(xi: float, alpha: float, w: np.ndarray) -> np.ndarray:
    """c = xi w / (1 + (xi - alpha) w): (N_bar^-1 + xi^-1)^-1 N_bar^-1 with N_bar = 1/w - alpha."""
    return xi * w / (1.0 + (xi - alpha) * w)


def cauchy_ratio(num: float, den: float) -> float:
    if den > 0.0:
        return math.sqrt(num / den)
    return 0.0 if num == 0.0 else math.inf


def iterate(T, a, r, f_alm, c, d, s_prev):
    """One iteration: harmonic step, synthesis, Cauchy sums, pixel step.

    Returns (a, s, r_next, sum (s - s_prev)^2, sum s^2).
    """
    at = T.omega * T.adjoint(r)
    a = f_alm[:, None] * (a + at)
    s = T.synth(a)
    num = float(np.sum((s - s_prev) ** 2))
    den = float(np.sum(s * s))
    r_next = c * (d - s)
    return a, s, r_next, num, den


@dataclass
class SolveResult:
    alm: np.ndarray
    map: np.ndarray
    xis: list
    ell_iters: list
    iters_per_level: list
    ratios: list = field(default_factory=list)
    converged: bool = True
    alpha: float = 0.0

    @property
    def n_iter(self):
        return int(sum(self.iters_per_level))


def solve(T, d, w, cl, beta=0.75, mu0=None, eps_final=1e-6, eps_coarse=1e-4,
          max_iter=1_000_000, replay=None, alm0=None, start_final=False) -> SolveResult:
    """Run the dual messenger to convergence (or for `replay[k]` iterations on level k).

    T supplies synth(a), adjoint(map), omega, npix and ell() (l of each
    coefficient slot).  With `start_final` only the xi = alpha level runs,
    starting from `alm0`, and the first residual is the pixel step applied to
    Y alm0.
    """
    d = np.asarray(d, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cl = np.asarray(cl, dtype=np.float64)
    alpha = alpha_of(w)
    sigma = 1.0 / T.omega
    ell = T.ell()
    xis = [alpha] if start_final else level_schedule(alpha, sigma, cl, beta, mu0)
    if replay is not None and len(replay) != len(xis):
        raise ValueError("replay has %d levels, schedule has %d" % (len(replay), len(xis)))
    if alm0 is None:
        a = np.zeros((ell.size, 2))
        s_prev = np.zeros_like(d)
        r = np.where(w > 0.0, d, 0.0)
    else:
        a = np.array(alm0, dtype=np.float64).reshape(ell.size, 2)
        s_prev = T.synth(a)
        r = pixel_coeff(xis[0], alpha, w) * (d - s_prev)
    res = SolveResult(a, s_prev, list(xis), [], [], alpha=alpha)
    total = 0
    for k, xi in enumerate(xis):
        mu, f, ell_iter = level_params(xi, alpha, sigma, cl)
        f_alm = f[ell]
        c = pixel_coeff(xi, alpha, w)
        eps = eps_final if xi <= alpha else eps_coarse
        it = 0
        while True:
            a, s, r, num, den = iterate(T, a, r, f_alm, c, d, s_prev)
            s_prev = s
            it += 1
            total += 1
            ratio = cauchy_ratio(num, den)
            res.ratios.append(ratio)
            if replay is not None:
                if it >= replay[k]:
                    break
            elif ratio < eps:
                break
            if total >= max_iter:
                res.converged = False
                break
        res.ell_iters.append(ell_iter)
        res.iters_per_level.append(it)
        if not res.converged:
            break
    res.alm, res.map = a, s_prev
    return res


def wf_residual(T, a, d, w, cl) -> float:
    """||A x - y|| / ||y|| for A = 1 + C^1/2 Y^H W Y C^1/2, x = C^-1/2 a, y = C^1/2 Y^H W d.

    The consistency check of the paper's Section 4 (the PCG form of the Wiener
    filter equation, Appendix C), restricted to modes with C_l > 0.
    """
    ell = T.ell()
    cla = np.asarray(cl)[ell]
    act = cla > 0.0
    sq = np.sqrt(np.where(act, cla, 0.0))[:, None]
    inv = np.where(act, 1.0 / np.sqrt(np.where(act, cla, 1.0)), 0.0)[:, None]
    s = T.synth(a)
    g = T.adjoint(w * (d - s))
    y = sq * T.adjoint(w * d)
    res = inv * a - sq * g
    res[~act] = 0.0
    y[~act] = 0.0
    return math.sqrt(T.dot(res, res) / T.dot(y, y))


def chi2(T, a, d, w, cl) -> float:
    """Posterior chi^2 = sum_p w (d - Y a)^2 + a^H C^-1 a over modes with C_l > 0."""
    ell = T.ell()
    cla = np.asarray(cl)[ell]
    act = cla > 0.0
    s = T.synth(a)
    pix = float(np.sum(w * (d - s) ** 2))
    b = np.where(act, 1.0 / np.where(act, cla, 1.0), 0.0)[:, None] * a
    return pix + T.dot(a, b)
