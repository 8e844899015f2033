"""Python binding of the C ABI in include/dmwf.h (argument marshalling only).

Every computation runs in the HIP library libdmwf.so built next to this file;
there is no fallback.  Arrays are torch tensors on the GPU (float64,
contiguous); the library enqueues its work on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmwf.so")

FP64, FP32_GEMM, BF16X3_GEMM = 0, 1, 2  # dmwf_precision: form of the Legendre contractions

STATUS = {0: "ok", 1: "invalid argument", 2: "workspace", 3: "HIP error", 4: "not converged",
          5: "non-finite", 6: "unsupported", 7: "out of memory"}
OK, ERR_INVALID_ARG, ERR_WORKSPACE, ERR_HIP, ERR_NOT_CONVERGED, ERR_NONFINITE, ERR_UNSUPPORTED, \
    ERR_OOM = range(8)


class DmwfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")
        self.status = status


class _PlanDesc(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int), ("lmax", ctypes.c_int), ("nmaps", ctypes.c_int),
                ("precision", ctypes.c_int)]


class _Schedule(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mu0", ctypes.c_double),
                ("eps_final", ctypes.c_double), ("eps_coarse", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("start_final", ctypes.c_int),
                ("replay_iters", ctypes.POINTER(ctypes.c_int)), ("n_replay", ctypes.c_int),
                ("want_residual", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("eps_reduced", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("n_iter", ctypes.c_int), ("alpha", ctypes.c_double),
                ("final_cauchy", ctypes.c_double), ("wf_residual", ctypes.c_double),
                ("cap_levels", ctypes.c_int), ("iters_per_level", ctypes.POINTER(ctypes.c_int)),
                ("xi_per_level", ctypes.POINTER(ctypes.c_double)),
                ("lmax_per_level", ctypes.POINTER(ctypes.c_int)), ("iters_reduced", ctypes.c_int)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libdmwf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(or python paper_1702_08852_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, ci, cd = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    lib.dmwf_plan_create.argtypes = [ctypes.POINTER(_PlanDesc), ctypes.POINTER(vp)]
    lib.dmwf_plan_destroy.argtypes = [vp]
    lib.dmwf_plan_destroy.restype = None
    lib.dmwf_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.dmwf_alm2map.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.dmwf_alm2map_static.argtypes = [vp, vp, vp, vp]
    lib.dmwf_adjoint.argtypes = [vp, vp, vp, ci, vp, sz, vp]
    lib.dmwf_dm_iterate.argtypes = [vp, cd, cd, vp, vp, vp, vp, vp, vp, ci, vp, sz, vp]
    lib.dmwf_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(_Schedule), vp, vp,
                               ctypes.POINTER(_Stats), vp, sz, vp]
    P = ctypes.POINTER
    lib.dmwf_solve_plans.argtypes = [ci, P(vp), P(vp), P(vp), P(vp), P(_Schedule), P(vp), P(vp),
                                     P(P(_Stats)), P(vp), P(sz), vp]
    lib.dmwf_legendre_work.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_longlong)]
    lib.dmwf_autotune.argtypes = [vp, vp, sz, vp, ctypes.POINTER(ci), ctypes.POINTER(ctypes.c_float)]
    lib.dmwf_set_tiles.argtypes = [vp, ci, ci, ci, ci]
    lib.dmwf_set_pipeline.argtypes = [vp, ci]
    lib.dmwf_pipeline_groups.argtypes = [vp]
    lib.dmwf_pipeline_groups.restype = ci
    lib.dmwf_wf_residual.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(cd), vp, sz, vp]
    lib.dmwf_profile_enable.argtypes = [vp, ci]
    lib.dmwf_profile_read.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_long), ctypes.POINTER(cd)]
    fp = ctypes.c_void_p
    lib.dmwf_nn_param_count.restype = ci
    lib.dmwf_nn_create.argtypes = [ci, ctypes.POINTER(vp)]
    lib.dmwf_nn_destroy.argtypes = [vp]
    lib.dmwf_nn_destroy.restype = None
    lib.dmwf_nn_get_params.argtypes = [vp, fp, vp]
    lib.dmwf_nn_set_params.argtypes = [vp, fp, vp]
    lib.dmwf_nn_noise_stats.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(cd),
                                        ctypes.POINTER(cd), vp]
    lib.dmwf_nn_features.argtypes = [ci, vp, vp, cd, cd, vp, ci, vp, fp, fp, vp]
    lib.dmwf_nn_forward.argtypes = [vp, fp, ci, fp, vp]
    lib.dmwf_nn_gradient.argtypes = [vp, fp, fp, ci, fp, fp, vp]
    lib.dmwf_nn_train_step.argtypes = [vp, fp, fp, ci, ctypes.c_float, fp, vp]
    lib.dmwf_nn_warm_start.argtypes = [vp, ci, vp, vp, cd, cd, vp, vp]
    lib.dmwf_status_string.argtypes = [ci]
    lib.dmwf_status_string.restype = ctypes.c_char_p
    lib.dmwf_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, where: str, allow=()):
    if status != OK and status not in allow:
        raise DmwfError(status, where, load().dmwf_last_error().decode())
    return status


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def n_alm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


@dataclass
class SolveStats:
    n_levels: int
    n_iter: int
    alpha: float
    final_cauchy: float
    wf_residual: float
    iters_per_level: list = field(default_factory=list)
    xi_per_level: list = field(default_factory=list)
    lmax_per_level: list = field(default_factory=list)
    status: int = OK
    iters_reduced: int = 0


class Plan:
    """A transform/solver plan for maps of one (nside, lmax), owning its workspace."""

    def __init__(self, nside: int, lmax: int, nmaps: int = 1, device=None, precision: int = FP64):
        lib = load()
        self.nside, self.lmax, self.nmaps = int(nside), int(lmax), int(nmaps)
        self.precision = int(precision)
        self.npix = 12 * self.nside * self.nside
        self.nalm = n_alm(self.lmax)
        dev = torch.device("cuda" if device is None else device)
        with torch.cuda.device(dev):
            h = ctypes.c_void_p()
            desc = _PlanDesc(self.nside, self.lmax, self.nmaps, self.precision)
            _check(lib.dmwf_plan_create(ctypes.byref(desc), ctypes.byref(h)), "dmwf_plan_create")
            self._h = h
            nb = ctypes.c_size_t()
            _check(lib.dmwf_workspace_bytes(self._h, ctypes.byref(nb)), "dmwf_workspace_bytes")
            self.ws_bytes = int(nb.value)
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.device = dev

    def close(self):
        if getattr(self, "_h", None):
            load().dmwf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --
    def _alm(self, out=None):
        if out is None:
            out = torch.empty((self.nmaps, self.nalm, 2) if self.nmaps > 1 else (self.nalm, 2),
                              dtype=torch.float64, device=self.device)
        return out

    def _map(self, out=None):
        if out is None:
            out = torch.empty((self.nmaps, self.npix) if self.nmaps > 1 else (self.npix,),
                              dtype=torch.float64, device=self.device)
        return out

    # -- entry points --
    def alm2map(self, alm: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._map(out)
        _check(load().dmwf_alm2map(self._h, _ptr(alm), _ptr(out), self.ws.data_ptr(),
                                   self.ws_bytes, _stream()), "dmwf_alm2map")
        return out

    def alm2map_static(self, alm: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """dmwf_alm2map_static: the synthesis with the library's fixed device
        scratch instead of this plan's workspace (allocates nothing)."""
        out = self._map(out)
        _check(load().dmwf_alm2map_static(self._h, _ptr(alm), _ptr(out), _stream()),
               "dmwf_alm2map_static")
        return out

    def adjoint(self, mp: torch.Tensor, scale_by_pixel_area: bool = False,
                out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._alm(out)
        _check(load().dmwf_adjoint(self._h, _ptr(mp), _ptr(out), int(bool(scale_by_pixel_area)),
                                   self.ws.data_ptr(), self.ws_bytes, _stream()), "dmwf_adjoint")
        return out

    def dm_iterate(self, xi: float, alpha: float, cl, d, ninv, alm_state, s_map, cauchy2,
                   first: bool) -> None:
        _check(load().dmwf_dm_iterate(self._h, float(xi), float(alpha), _ptr(cl), _ptr(d),
                                      _ptr(ninv), _ptr(alm_state), _ptr(s_map), _ptr(cauchy2),
                                      int(bool(first)), self.ws.data_ptr(), self.ws_bytes,
                                      _stream()), "dmwf_dm_iterate")

    def solve(self, cl, d, ninv, beta: float = 0.75, mu0: float = -1.0, eps_final: float = 1e-6,
              eps_coarse: float = 1e-4, max_iter: int = 1_000_000, replay=None,
              start_final: bool = False, alm: torch.Tensor | None = None,
              out_map: torch.Tensor | None = None, want_residual: bool = False,
              raise_on_cap: bool = False, cap_levels: int = 512, eps_reduced: float = -1.0,
              warm_start: bool = False):
        """dmwf_solve.  start_final / warm_start: alm holds the starting a_lm
        (the last level only, or the whole cooling schedule)."""
        alm = self._alm(alm)
        out_map = self._map(out_map)
        sc, keep = _schedule(beta, mu0, eps_final, eps_coarse, max_iter, replay, start_final,
                             want_residual, eps_reduced, warm_start)
        sts, bufs = _stats(self.nmaps, cap_levels)
        status = load().dmwf_solve(self._h, _ptr(cl), _ptr(d), _ptr(ninv), ctypes.byref(sc),
                                   _ptr(alm), _ptr(out_map), sts,
                                   self.ws.data_ptr(), self.ws_bytes, _stream())
        _check(status, "dmwf_solve", allow=() if raise_on_cap else (ERR_NOT_CONVERGED,))
        out = _read_stats(sts, bufs, cap_levels, status)
        return alm, out_map, (out[0] if self.nmaps == 1 else out)

    def autotune(self):
        """Time the Legendre tiles on this plan's shape and keep the fastest.
        Returns ((synthesis rings per lane, synthesis maps per wave, analysis
        rings per lane, analysis maps per wave), {candidate: ms})."""
        ch = (ctypes.c_int * 4)()
        ms = (ctypes.c_float * 12)()
        _check(load().dmwf_autotune(self._h, self.ws.data_ptr(), self.ws_bytes, _stream(), ch, ms),
               "dmwf_autotune")
        times = {f"syn{1 + i // 4}x{1 << (i % 4)}": float(ms[i]) for i in range(8) if ms[i] >= 0.0}
        times.update({f"ana{4 if t < 2 else 8}x{1 + (t & 1)}": float(ms[8 + t])
                      for t in range(4) if ms[8 + t] >= 0.0})
        return (int(ch[0]), int(ch[1]), int(ch[2]), int(ch[3])), times

    def legendre_work(self, ell: int) -> dict:
        """dmwf_legendre_work: full, started and issued triples of one FP64
        Legendre launch at band limit ell."""
        out = (ctypes.c_longlong * 4)()
        _check(load().dmwf_legendre_work(self._h, int(ell), out), "dmwf_legendre_work")
        return {"full": out[0], "started": out[1], "synthesis_issued": out[2],
                "analysis_issued": out[3]}

    def set_tiles(self, syn_k: int, syn_mb: int, ana_k: int, ana_mb: int = 1) -> None:
        _check(load().dmwf_set_tiles(self._h, int(syn_k), int(syn_mb), int(ana_k), int(ana_mb)),
               "dmwf_set_tiles")

    def set_pipeline(self, groups: int) -> None:
        """dmwf_set_pipeline, kept for ABI stability: the pipelined iteration
        is not built, so only 0 and 1 (off) are accepted; 2..8 raise with
        DMWF_ERR_UNSUPPORTED."""
        _check(load().dmwf_set_pipeline(self._h, int(groups)), "dmwf_set_pipeline")

    @property
    def pipeline_groups(self) -> int:
        return int(load().dmwf_pipeline_groups(self._h))

    def wf_residual(self, cl, d, ninv, alm):
        """FP64 residual of the Wiener filter system: a float for a one-map
        plan, a list of nmaps floats otherwise."""
        out = (ctypes.c_double * self.nmaps)()
        _check(load().dmwf_wf_residual(self._h, _ptr(cl), _ptr(d), _ptr(ninv), _ptr(alm),
                                       out, self.ws.data_ptr(), self.ws_bytes,
                                       _stream()), "dmwf_wf_residual")
        vals = [float(v) for v in out]
        return vals[0] if self.nmaps == 1 else vals

    def profile(self, enable=True) -> None:
        """True or 1: time every launch; 2: time the Legendre analysis launches
        only (the solve loop keeps replaying the rest from its graph); False
        or 0: off."""
        level = enable if isinstance(enable, int) and not isinstance(enable, bool) else int(bool(enable))
        _check(load().dmwf_profile_enable(self._h, level), "dmwf_profile_enable")

    def profile_read(self) -> dict:
        n = ctypes.c_int()
        names = (ctypes.c_char_p * 16)()
        counts = (ctypes.c_long * 16)()
        ms = (ctypes.c_double * 16)()
        _check(load().dmwf_profile_read(self._h, ctypes.byref(n), names, counts, ms),
               "dmwf_profile_read")
        return {names[i].decode(): (int(counts[i]), float(ms[i])) for i in range(n.value)}


def _schedule(beta, mu0, eps_final, eps_coarse, max_iter, replay, start_final, want_residual,
              eps_reduced, warm_start=False):
    rep = None
    if replay is not None:
        rep = (ctypes.c_int * len(replay))(*[int(v) for v in replay])
    sc = _Schedule(float(beta), float(mu0), float(eps_final), float(eps_coarse),
                   int(max_iter), int(bool(start_final)),
                   ctypes.cast(rep, ctypes.POINTER(ctypes.c_int)) if rep is not None else None,
                   len(replay) if replay is not None else 0, int(bool(want_residual)),
                   int(bool(warm_start)), float(eps_reduced))
    return sc, rep


def _stats(nm, cap_levels):
    bufs = [((ctypes.c_int * cap_levels)(), (ctypes.c_double * cap_levels)(),
             (ctypes.c_int * cap_levels)()) for _ in range(nm)]
    sts = (_Stats * nm)(*[_Stats(0, 0, 0.0, 0.0, -1.0, cap_levels, *b, 0) for b in bufs])
    return sts, bufs


def _read_stats(sts, bufs, cap_levels, status):
    out = []
    for st, (ipl, xpl, lpl) in zip(sts, bufs):
        nl = min(st.n_levels, cap_levels)
        out.append(SolveStats(st.n_levels, st.n_iter, st.alpha, st.final_cauchy,
                              st.wf_residual, list(ipl[:nl]), list(xpl[:nl]),
                              list(lpl[:nl]), status, st.iters_reduced))
    return out


def solve_plans(plans, cls, ds, ninvs, beta: float = 0.75, mu0: float = -1.0,
                eps_final: float = 1e-6, eps_coarse: float = 1e-4, max_iter: int = 1_000_000,
                replay=None, want_residual: bool = False, raise_on_cap: bool = False,
                cap_levels: int = 512, eps_reduced: float = -1.0):
    """dmwf_solve_plans: every plan's maps solved together (one graph for all
    plans' iterations).  Returns [(alm, map, stats)] per plan, stats as
    Plan.solve returns them."""
    n = len(plans)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    alms = [pl._alm() for pl in plans]
    maps = [pl._map() for pl in plans]
    arr = lambda xs: (vp * n)(*xs)
    sc, keep = _schedule(beta, mu0, 0.0 + eps_final, eps_coarse, max_iter, replay, False,
                         want_residual, eps_reduced)
    st_bufs = [_stats(pl.nmaps, cap_levels) for pl in plans]
    st_ptrs = (P(_Stats) * n)(*[ctypes.cast(sb[0], P(_Stats)) for sb in st_bufs])
    wsb = (ctypes.c_size_t * n)(*[pl.ws_bytes for pl in plans])
    status = load().dmwf_solve_plans(
        n, arr([pl._h.value for pl in plans]), arr([_ptr(x) for x in cls]),
        arr([_ptr(x) for x in ds]), arr([_ptr(x) for x in ninvs]), ctypes.byref(sc),
        arr([_ptr(x) for x in alms]), arr([_ptr(x) for x in maps]), st_ptrs,
        arr([pl.ws.data_ptr() for pl in plans]), wsb, _stream())
    _check(status, "dmwf_solve_plans", allow=() if raise_on_cap else (ERR_NOT_CONVERGED,))
    res = []
    for pl, a, m, (sts, bufs) in zip(plans, alms, maps, st_bufs):
        out = _read_stats(sts, bufs, cap_levels, status)
        res.append((a, m, out[0] if pl.nmaps == 1 else out))
    return res


def _fptr(t):
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 CUDA tensor")
    return t.data_ptr()


def _iptr(t):
    if t is None:
        return None
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("expected a contiguous int32 CUDA tensor")
    return t.data_ptr()


N_FEATURES, N_OUT = 24, 2


class Net:
    """The warm-start network (dmwf_nn): FP32 parameters on the device."""

    def __init__(self, max_batch: int = 65536, device=None):
        lib = load()
        dev = torch.device("cuda" if device is None else device)
        with torch.cuda.device(dev):
            h = ctypes.c_void_p()
            _check(lib.dmwf_nn_create(int(max_batch), ctypes.byref(h)), "dmwf_nn_create")
        self._h, self.device, self.max_batch = h, dev, int(max_batch)
        self.n_params = int(lib.dmwf_nn_param_count())

    def close(self):
        if getattr(self, "_h", None):
            load().dmwf_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(load().dmwf_nn_get_params(self._h, _fptr(out), _stream()), "dmwf_nn_get_params")
        return out

    def set_params(self, p: torch.Tensor) -> None:
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(load().dmwf_nn_set_params(self._h, _fptr(p), _stream()), "dmwf_nn_set_params")

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        n = x.shape[0]
        y = torch.empty((n, N_OUT), dtype=torch.float32, device=self.device)
        _check(load().dmwf_nn_forward(self._h, _fptr(x), n, _fptr(y), _stream()), "dmwf_nn_forward")
        return y

    def gradient(self, x: torch.Tensor, t: torch.Tensor):
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(load().dmwf_nn_gradient(self._h, _fptr(x), _fptr(t), x.shape[0], _fptr(g),
                                       _fptr(loss), _stream()), "dmwf_nn_gradient")
        return g, loss

    def train_step(self, x: torch.Tensor, t: torch.Tensor, lr: float, loss: torch.Tensor):
        _check(load().dmwf_nn_train_step(self._h, _fptr(x), _fptr(t), x.shape[0], float(lr),
                                         _fptr(loss), _stream()), "dmwf_nn_train_step")

    def warm_start(self, lmax: int, dlm: torch.Tensor, cl: torch.Tensor, noise_w: float,
                   fsky: float) -> torch.Tensor:
        out = torch.empty((n_alm(lmax), 2), dtype=torch.float64, device=self.device)
        _check(load().dmwf_nn_warm_start(self._h, int(lmax), _ptr(dlm), _ptr(cl), float(noise_w),
                                         float(fsky), _ptr(out), _stream()), "dmwf_nn_warm_start")
        return out


def noise_stats(ninv: torch.Tensor):
    """(N_w, sky fraction) of one map: dmwf_nn_noise_stats."""
    nw, fs = ctypes.c_double(), ctypes.c_double()
    _check(load().dmwf_nn_noise_stats(_ptr(ninv), ninv.numel(), ctypes.byref(nw), ctypes.byref(fs),
                                      _stream()), "dmwf_nn_noise_stats")
    return nw.value, fs.value


def nn_features(lmax: int, dlm: torch.Tensor, cl: torch.Tensor, noise_w: float, fsky: float,
                slots: torch.Tensor | None = None, n: int | None = None,
                target: torch.Tensor | None = None):
    """Feature rows (and targets) of the listed a_lm slots: dmwf_nn_features."""
    n = int(slots.numel()) if slots is not None else int(n if n is not None else n_alm(lmax))
    x = torch.empty((n, N_FEATURES), dtype=torch.float32, device=dlm.device)
    t = torch.empty((n, N_OUT), dtype=torch.float32, device=dlm.device) if target is not None else None
    _check(load().dmwf_nn_features(int(lmax), _ptr(dlm), _ptr(cl), float(noise_w), float(fsky),
                                   _iptr(slots), n, _ptr(target), _fptr(x), _fptr(t), _stream()),
           "dmwf_nn_features")
    return x, t


def status_string(status: int) -> str:
    return load().dmwf_status_string(status).decode()
