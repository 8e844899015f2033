"""CPU oracle for the dual messenger Wiener filter on the HEALPix sphere.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import or call anything in this package.
The product library never touches it and it never touches the product: the
two share no code, tables or helpers.

Contents
  sht.c     plain FP64 synthesis / adjoint on the ring grid (direct sums)
  dm.py     the dual messenger iteration (paper Algorithm 2, hybrid form with
            cooling of xi), written on the sphere in residual form
  dense.py  the Wiener filter equation solved as a dense linear system
            (small Nside only), and the fixed point of one cooling level

Every routine is FP64.  Where the paper is silent or ambiguous the reading
taken is stated in the docstring concerned.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile sht.c with gcc into oracle/_build/liboracle.so."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, os.path.join(_HERE, "sht.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        L = ctypes.POINTER(ctypes.c_long)
        ci, cd = ctypes.c_int, ctypes.c_double
        lib.or_ring.argtypes = [ci, ci, D, D, L, D, L]
        lib.or_lognorm.argtypes = [ci]
        lib.or_lognorm.restype = cd
        lib.or_lambda_scaled.argtypes = [ci, cd, cd, ci, D, I]
        lib.or_lambda.argtypes = [ci, cd, cd, ci, D]
        lib.or_alm2map.argtypes = [ci, ci, D, D, ci]
        lib.or_alm2map_rings.argtypes = [ci, ci, D, I, ci, D, ci]
        lib.or_adjoint.argtypes = [ci, ci, D, D, ci]
        lib.or_adjoint_m.argtypes = [ci, ci, D, I, ci, D, ci]
        lib.or_max_threads.restype = ci
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def max_threads() -> int:
    return int(_load().or_max_threads())


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------
def npix(nside: int) -> int:
    return 12 * nside * nside


def n_alm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(l, m, lmax):
    return m * (2 * lmax + 1 - m) // 2 + l


def ring(nside: int, r: int):
    """(z, sin theta, nph, phi0, first pixel) of ring r = 1..4N-1."""
    lib = _load()
    z, st, p0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n, s = ctypes.c_long(), ctypes.c_long()
    lib.or_ring(nside, r, ctypes.byref(z), ctypes.byref(st), ctypes.byref(n),
                ctypes.byref(p0), ctypes.byref(s))
    return z.value, st.value, n.value, p0.value, s.value


def rings(nside: int):
    """Arrays over rings 1..4N-1: z, sin theta, nph, phi0, start."""
    rs = [ring(nside, r) for r in range(1, 4 * nside)]
    z, st, n, p0, s = (np.array(v) for v in zip(*rs))
    return z, st, n.astype(np.int64), p0, s.astype(np.int64)


def pixel_angles(nside: int):
    """theta, phi of every pixel in RING order."""
    z, st, n, p0, s = rings(nside)
    th = np.empty(npix(nside))
    ph = np.empty(npix(nside))
    for k in range(len(z)):
        th[s[k]:s[k] + n[k]] = math.atan2(st[k], z[k])
        ph[s[k]:s[k] + n[k]] = p0[k] + 2.0 * math.pi * np.arange(n[k]) / n[k]
    return th, ph


# ---------------------------------------------------------------------------
# Associated Legendre functions (normalised, Condon-Shortley phase)
# ---------------------------------------------------------------------------
def lambda_lm(m: int, x: float, sint: float, lmax: int) -> np.ndarray:
    """lambda_lm(x) for l = m..lmax; Y_lm = lambda_lm(cos theta) e^{i m phi}."""
    out = np.zeros(max(lmax - m + 1, 0))
    if out.size:
        _load().or_lambda(m, float(x), float(sint), lmax, _dp(out))
    return out


def lambda_lm_scaled(m: int, x: float, sint: float, lmax: int):
    """(mantissa, binary exponent) of lambda_lm for l = m..lmax."""
    cnt = max(lmax - m + 1, 0)
    mt = np.zeros(cnt)
    ex = np.zeros(cnt, dtype=np.int32)
    if cnt:
        _load().or_lambda_scaled(m, float(x), float(sint), lmax, _dp(mt), _ip(ex))
    return mt, ex


def lognorm(m: int) -> float:
    return float(_load().or_lognorm(m))


# ---------------------------------------------------------------------------
# Transforms
# ---------------------------------------------------------------------------
def alm2map(alm: np.ndarray, nside: int, lmax: int, nthreads: int = 0) -> np.ndarray:
    """s_p = sum_lm a_lm Y_lm(p) (real field), alm [n_alm, 2] m-major."""
    a = np.ascontiguousarray(alm, dtype=np.float64).reshape(n_alm(lmax), 2)
    out = np.zeros(npix(nside))
    _load().or_alm2map(nside, lmax, _dp(a), _dp(out), nthreads)
    return out


def alm2map_rings(alm: np.ndarray, nside: int, lmax: int, ring_list, nthreads: int = 0):
    """Synthesis on the listed rings only; returns the concatenated ring values."""
    a = np.ascontiguousarray(alm, dtype=np.float64).reshape(n_alm(lmax), 2)
    rl = np.ascontiguousarray(ring_list, dtype=np.int32)
    tot = sum(ring(nside, int(r))[2] for r in rl)
    out = np.zeros(tot)
    _load().or_alm2map_rings(nside, lmax, _dp(a), _ip(rl), len(rl), _dp(out), nthreads)
    return out


def adjoint(mp: np.ndarray, nside: int, lmax: int, nthreads: int = 0) -> np.ndarray:
    """b_lm = sum_p map_p conj(Y_lm(p)) (no pixel-area factor), [n_alm, 2]."""
    v = np.ascontiguousarray(mp, dtype=np.float64)
    out = np.zeros((n_alm(lmax), 2))
    _load().or_adjoint(nside, lmax, _dp(v), _dp(out), nthreads)
    return out


def adjoint_m(mp: np.ndarray, nside: int, lmax: int, ms, nthreads: int = 0):
    """The adjoint for the listed m only: dict m -> [lmax-m+1, 2] over l = m..lmax."""
    v = np.ascontiguousarray(mp, dtype=np.float64)
    msa = np.ascontiguousarray(ms, dtype=np.int32)
    tot = int(sum(lmax - int(m) + 1 for m in msa))
    out = np.zeros((tot, 2))
    _load().or_adjoint_m(nside, lmax, _dp(v), _ip(msa), len(msa), _dp(out), nthreads)
    res, o = {}, 0
    for m in msa:
        c = lmax - int(m) + 1
        res[int(m)] = out[o:o + c].copy()
        o += c
    return res


def alm_dot(a: np.ndarray, b: np.ndarray, lmax: int) -> float:
    """Real inner product on a_lm counting m > 0 twice (the sphere's L2 on real fields)."""
    wgt = np.full(n_alm(lmax), 2.0)
    wgt[:lmax + 1] = 1.0
    return float(np.sum(wgt * (a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1])))


def ell_of_index(lmax: int) -> np.ndarray:
    """l for every m-major alm slot."""
    return np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])


def m_of_index(lmax: int) -> np.ndarray:
    return np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])


class SphereTransforms:
    """F^-1 = Y (synthesis) and F = Omega Y^H on the HEALPix grid, via the oracle."""

    def __init__(self, nside: int, lmax: int, nthreads: int = 0):
        self.nside, self.lmax, self.nthreads = nside, lmax, nthreads
        self.npix = npix(nside)
        self.omega = 4.0 * math.pi / self.npix

    def synth(self, alm):
        return alm2map(alm, self.nside, self.lmax, self.nthreads)

    def adjoint(self, mp):
        return adjoint(mp, self.nside, self.lmax, self.nthreads)

    def ell(self):
        return ell_of_index(self.lmax)

    def dot(self, a, b):
        return alm_dot(a, b, self.lmax)


from . import dm, dense  # noqa: E402,F401
