"""Seeded synthetic workloads for the dual messenger Wiener filter on the sphere.

This module only draws random numbers and lays them out on the HEALPix ring
grid: signal harmonic coefficients with a prescribed angular power spectrum,
per-pixel noise levels, unit white noise and sky masks.  It holds none of the
method's arithmetic (no spherical harmonic transform, no Wiener filter step),
so the GPU path and the CPU oracle can both be fed from it without sharing any
code.  The data map d = Y a + n needs a synthesis Y; the caller supplies it
(`data_map`).

The paper's only experiment uses a CAMB spectrum on a flat 512^2 patch
(Section 3), which is not reproduced here.  These recipes stand in for it on
the sphere: an analytic C_l, inhomogeneous noise and a galactic cut plus point
source holes, at the sizes of the three single-map configurations below.

Every draw is reproducible from (config id, map index, stream name).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 170208852

# Ecliptic north pole in galactic coordinates (l, b) in degrees.  Only the
# tilt (about 60 degrees from the galactic pole) shapes the noise pattern.
ECLIPTIC_POLE_LB = (96.38, 29.81)


def _rng(config: int, index: int, stream: str) -> np.random.Generator:
    tag = sum((i + 1) * ord(c) for i, c in enumerate(stream))
    ss = np.random.SeedSequence([SEED_BASE + 1000 * config + index, tag])
    return np.random.default_rng(ss)


# ---------------------------------------------------------------------------
# HEALPix ring layout (Gorski et al. 2005, RING scheme), used here only to
# place masks and noise on pixels.
# ---------------------------------------------------------------------------
def ring_layout(nside: int):
    """Per-ring (z, nph, phi of first pixel, first pixel index), rings 1..4N-1."""
    n = nside
    nr = 4 * n - 1
    z = np.empty(nr)
    nph = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    start = np.empty(nr, dtype=np.int64)
    npix = 12 * n * n
    for k in range(nr):
        i = k + 1
        if i < n:
            z[k] = 1.0 - i * i / (3.0 * n * n)
            nph[k] = 4 * i
            phi0[k] = math.pi / (4.0 * i)
            start[k] = 2 * i * (i - 1)
        elif i <= 3 * n:
            z[k] = 4.0 / 3.0 - 2.0 * i / (3.0 * n)
            nph[k] = 4 * n
            s = (i - n + 1) % 2
            phi0[k] = math.pi / (2.0 * n) * (s / 2.0)
            start[k] = 2 * n * (n - 1) + 4 * n * (i - n)
        else:
            j = 4 * n - i
            z[k] = -(1.0 - j * j / (3.0 * n * n))
            nph[k] = 4 * j
            phi0[k] = math.pi / (4.0 * j)
            start[k] = npix - 2 * j * (j + 1)
    return z, nph, phi0, start


def pixel_centres(nside: int):
    """(theta, phi) of every pixel in RING order."""
    z, nph, phi0, start = ring_layout(nside)
    npix = 12 * nside * nside
    theta = np.empty(npix)
    phi = np.empty(npix)
    for k in range(len(z)):
        s, c = start[k], nph[k]
        theta[s:s + c] = math.acos(z[k])
        phi[s:s + c] = phi0[k] + 2.0 * math.pi * np.arange(c) / c
    return theta, phi


def _unit_vectors(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=1)


# ---------------------------------------------------------------------------
# Spectra
# ---------------------------------------------------------------------------
def cl_inverse_square(lmax: int) -> np.ndarray:
    """C_l = 1/(l(l+1)) for l >= 2, zero for l < 2."""
    cl = np.zeros(lmax + 1)
    l = np.arange(2, lmax + 1, dtype=np.float64)
    cl[2:] = 1.0 / (l * (l + 1.0))
    return cl


def cl_damped(lmax: int, amp: float = 2.0 * math.pi * 1e3, lcut: float = 400.0) -> np.ndarray:
    """C_l = amp/(l(l+1)) exp(-(l/lcut)^2) [uK^2] for l >= 2, zero below."""
    cl = np.zeros(lmax + 1)
    l = np.arange(2, lmax + 1, dtype=np.float64)
    cl[2:] = amp / (l * (l + 1.0)) * np.exp(-(l / lcut) ** 2)
    return cl


def n_alm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def draw_alm(cl: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Gaussian a_lm with E|a_lm|^2 = C_l, m-major layout, shape [n_alm, 2].

    m = 0 entries are real N(0, C_l); m > 0 have Re, Im ~ N(0, C_l/2).
    """
    lmax = len(cl) - 1
    out = np.zeros((n_alm(lmax), 2))
    off = 0
    for m in range(lmax + 1):
        cnt = lmax + 1 - m
        c = cl[m:]
        if m == 0:
            out[off:off + cnt, 0] = rng.standard_normal(cnt) * np.sqrt(c)
        else:
            g = rng.standard_normal((cnt, 2))
            out[off:off + cnt] = g * np.sqrt(c / 2.0)[:, None]
        off += cnt
    return out


# ---------------------------------------------------------------------------
# Masks and noise
# ---------------------------------------------------------------------------
_TREES: dict = {}


def hole_mask(nside: int, n_holes: int, radius_deg: float, rng: np.random.Generator,
              vec: np.ndarray | None = None) -> np.ndarray:
    """Boolean map, True inside any of n_holes discs with centres uniform on the sphere."""
    from scipy.spatial import cKDTree

    npix = 12 * nside * nside
    if n_holes == 0:
        return np.zeros(npix, dtype=bool)
    cz = rng.uniform(-1.0, 1.0, n_holes)
    cphi = rng.uniform(0.0, 2.0 * math.pi, n_holes)
    centres = _unit_vectors(np.arccos(cz), cphi)
    chord = 2.0 * math.sin(math.radians(radius_deg) / 2.0)
    if vec is None:
        # the pixel-centre tree of an Nside is built once and reused
        tree = _TREES.get(nside)
        if tree is None:
            tree = _TREES[nside] = cKDTree(_unit_vectors(*pixel_centres(nside)))
    else:
        tree = cKDTree(vec)
    mask = np.zeros(npix, dtype=bool)
    for idx in tree.query_ball_point(centres, chord):
        mask[idx] = True
    return mask


def band_mask(nside: int, bcut_deg: float) -> np.ndarray:
    """True where |galactic latitude| < bcut (HEALPix z axis = galactic pole)."""
    theta, _ = pixel_centres(nside)
    return np.abs(np.cos(theta)) < math.sin(math.radians(bcut_deg))


def band_for_fraction(nside: int, holes: np.ndarray, fraction: float):
    """Smallest |b| cut whose union with `holes` masks at least `fraction` of the sky."""
    theta, _ = pixel_centres(nside)
    absz = np.abs(np.cos(theta))
    npix = absz.size
    need = int(round(fraction * npix)) - int(holes.sum())
    if need <= 0:
        return 0.0, holes.copy()
    free = np.sort(absz[~holes])
    zcut = free[min(need, free.size) - 1]
    mask = holes | (absz <= zcut)
    return math.degrees(math.asin(min(1.0, zcut))), mask


def ecliptic_cos2(nside: int) -> np.ndarray:
    """cos^2 of ecliptic latitude per pixel."""
    theta, phi = pixel_centres(nside)
    lp, bp = (math.radians(v) for v in ECLIPTIC_POLE_LB)
    pole = np.array([math.cos(bp) * math.cos(lp), math.cos(bp) * math.sin(lp), math.sin(bp)])
    sinb = _unit_vectors(theta, phi) @ pole
    return 1.0 - sinb * sinb


# ---------------------------------------------------------------------------
# Problems
# ---------------------------------------------------------------------------
@dataclass
class Problem:
    """One Wiener filter instance: spectrum, true a_lm, noise levels, mask."""
    name: str
    nside: int
    lmax: int
    cl: np.ndarray            # [lmax+1]
    alm_true: np.ndarray      # [n_alm, 2]
    sigma: np.ndarray         # [npix] per-pixel noise rms
    white: np.ndarray         # [npix] unit normal draws
    mask: np.ndarray          # [npix] bool, True = masked
    eps_final: float
    meta: dict = field(default_factory=dict)

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def ninv(self) -> np.ndarray:
        """Inverse noise variance per pixel, 0 on masked pixels."""
        w = 1.0 / (self.sigma * self.sigma)
        w[self.mask] = 0.0
        return w

    def data_map(self, signal_map: np.ndarray) -> np.ndarray:
        """d = signal + sigma * white on unmasked pixels, 0 on masked pixels."""
        d = signal_map + self.sigma * self.white
        d[self.mask] = 0.0
        return d


CONFIGS = {
    # name: (config id, default nside, lmax factor)
    "cfg1": 1,   # Nside 16, lmax 32: C_l = 1/(l(l+1)), lognormal noise, |b|<10 + 10 holes of 5 deg
    "cfg2": 2,   # Nside 256, lmax 512: damped spectrum, ecliptic hits, |b|<15 + 200 holes of 1 deg
    "cfg3": 3,   # Nside 1024, lmax 2048: as cfg2, sigma0 45 uK, 20% masked (band + 2000 holes of 0.3 deg)
    "cfg4": 4,   # batch member: damped spectrum, own |b| cut 5-20 deg + 50-500 holes of 1 deg,
                 # sigma0 ~ U[10, 60] uK times a lognormal(0, 0.25) per-pixel modulation
    "cfg5": 5,   # warm-start training / evaluation map: configuration 2's shape (|b| < 15
                 # + 200 holes of 1 deg, 30 uK ecliptic hits), its own holes and draws per index
}

DEFAULT_NSIDE = {"cfg1": 16, "cfg2": 256, "cfg3": 1024, "cfg4": 128, "cfg5": 256}

# Warm-start workload: training maps are cfg5 indices 0..1999 at Nside 256,
# evaluation maps the unseen indices from 100000 on at Nside 512.
WARM_TRAIN_NSIDE, WARM_TRAIN_MAPS = 256, 2000
WARM_EVAL_NSIDE, WARM_EVAL_MAPS, WARM_EVAL_FIRST = 512, 16, 100000

# The batched workload: maps per Nside (lmax = 2 Nside), 96 in all.
BATCH_GROUPS = ((128, 48), (256, 32), (512, 16))


def batch_members(nside: int):
    """Map indices of the batched workload that have this Nside (each member
    draws its own mask and noise from its index)."""
    start = 0
    for ns, cnt in BATCH_GROUPS:
        if ns == nside:
            return list(range(start, start + cnt))
        start += cnt
    raise KeyError(nside)


def make_problem(name: str, nside: int | None = None, lmax: int | None = None,
                 index: int = 0) -> Problem:
    """Build configuration `name` ("cfg1", "cfg2", "cfg3"), optionally at another Nside.

    The recipe (spectrum shape, noise model, mask model) is kept when Nside is
    changed, which gives the same workload structure at sizes the oracle can
    handle; lmax defaults to 2*Nside.
    """
    cid = CONFIGS[name]
    nside = DEFAULT_NSIDE[name] if nside is None else int(nside)
    lmax = 2 * nside if lmax is None else int(lmax)
    npix = 12 * nside * nside
    r_alm = _rng(cid, index, "alm")
    r_sig = _rng(cid, index, "sigma")
    r_wht = _rng(cid, index, "white")
    r_hol = _rng(cid, index, "holes")
    meta = {"config": cid, "index": index}
    if name == "cfg1":
        cl = cl_inverse_square(lmax)
        sigma = np.exp(r_sig.normal(0.0, 0.5, npix))
        mask = band_mask(nside, 10.0) | hole_mask(nside, 10, 5.0, r_hol)
        eps = 1e-8
        meta.update(bcut_deg=10.0, holes=10, hole_deg=5.0, noise="lognormal(0,0.5)")
    elif name in ("cfg2", "cfg3", "cfg5"):
        cl = cl_damped(lmax)
        sigma0 = 45.0 if name == "cfg3" else 30.0
        hits = 1.0 + 4.0 * ecliptic_cos2(nside)
        sigma = sigma0 / np.sqrt(hits)
        if name in ("cfg2", "cfg5"):
            mask = band_mask(nside, 15.0) | hole_mask(nside, 200, 1.0, r_hol)
            meta.update(bcut_deg=15.0, holes=200, hole_deg=1.0)
        else:
            holes = hole_mask(nside, 2000, 0.3, r_hol)
            bcut, mask = band_for_fraction(nside, holes, 0.20)
            meta.update(bcut_deg=bcut, holes=2000, hole_deg=0.3, hole_fraction=float(holes.mean()))
        eps = 1e-6
        meta.update(sigma0_uK=sigma0, noise="sigma0/sqrt(1+4cos^2(beta_ecl))")
    elif name == "cfg4":
        r_par = _rng(cid, index, "params")
        cl = cl_damped(lmax)
        sigma0 = float(r_par.uniform(10.0, 60.0))
        bcut = float(r_par.uniform(5.0, 20.0))
        nholes = int(r_par.integers(50, 501))
        sigma = sigma0 * np.exp(r_sig.normal(0.0, 0.25, npix))
        mask = band_mask(nside, bcut) | hole_mask(nside, nholes, 1.0, r_hol)
        eps = 1e-6
        meta.update(sigma0_uK=sigma0, bcut_deg=bcut, holes=nholes, hole_deg=1.0,
                    noise="sigma0*exp(N(0,0.25))")
    else:  # pragma: no cover
        raise KeyError(name)
    alm = draw_alm(cl, r_alm)
    white = r_wht.standard_normal(npix)
    meta["masked_fraction"] = float(mask.mean())
    return Problem(name, nside, lmax, cl, alm, sigma, white, mask, eps, meta)


def random_alm(lmax: int, seed: int, cl: np.ndarray | None = None) -> np.ndarray:
    """Test helper: Gaussian a_lm (flat spectrum unless cl given), Im a_l0 = 0."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 77, seed]))
    if cl is None:
        cl = np.ones(lmax + 1)
    return draw_alm(cl, rng)


def nn_init_params(seed: int) -> np.ndarray:
    """Initial parameters of the warm-start network (flat FP32, layout W1 [24][128],
    b1, W2 [128][128], b2, W3 [128][2], b3): He-normal weights, zero biases,
    the output layer scaled down by 10."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 79, seed]))
    parts = []
    for fan_in, fan_out, scale in ((24, 128, 1.0), (128, 128, 1.0), (128, 2, 0.1)):
        parts.append(rng.standard_normal(fan_in * fan_out) * math.sqrt(2.0 / fan_in) * scale)
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def random_map(nside: int, seed: int) -> np.ndarray:
    """Test helper: unit normal map."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 78, seed]))
    return rng.standard_normal(12 * nside * nside)
