"""ctypes binding of libesim.so (include/esim.h).

Argument marshalling only: every step of the event simulation runs in the HIP
kernels of libesim.  Tensors are torch CUDA (HIP) tensors; calls are enqueued
on the current torch stream unless a stream is given.  If the library is not
built this module raises at load time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesim.so")

MAX_F = 12
MAX_D = MAX_F + 2

OK, E_INVAL, E_HIP, E_CAPACITY, E_UNSUPPORTED = 0, -1, -2, -3, -4
F32, F16 = 0, 1
INIT, THRESHOLDED, EXHAUSTIVE, RAW = 0, 1, 2, 3
GRAM_F64, GRAM_F32C = 0, 1
THRESHOLD_CLOSED, THRESHOLD_LAST_WINDOW, THRESHOLD_NEW_WINDOW = 0, 1, 2


class EsimError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class esim_clip(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("T", ctypes.c_int32),
                ("F", ctypes.c_int32), ("feat_dtype", ctypes.c_int32),
                ("y", ctypes.c_void_p), ("feat", ctypes.c_void_p)]


class esim_params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("tr", ctypes.c_int32), ("C", ctypes.c_double),
                ("h", ctypes.c_double), ("b", ctypes.c_double * MAX_D),
                ("ridge", ctypes.c_double), ("precision", ctypes.c_int32),
                ("kappa_fp64", ctypes.c_double), ("multi_crossing", ctypes.c_int32),
                ("threshold", ctypes.c_int32), ("dt", ctypes.c_double)]


class esim_state(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("xref", ctypes.c_void_p), ("tref", ctypes.c_void_p), ("last", ctypes.c_void_p),
                ("bxy", ctypes.c_void_p), ("rmom", ctypes.c_void_p)]


class esim_events_buf(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("clip", ctypes.c_void_p),
                ("capacity", ctypes.c_int64), ("count", ctypes.c_void_p), ("ts", ctypes.c_void_p)]


# Every symbol the header declares, with (restype, argtypes).
_vp, _i32, _i64, _sz, _f32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                              ctypes.c_float)
SIGNATURES = {
    "esim_plan_create": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "esim_plan_destroy": (_i32, [_vp]),
    "esim_plan_pixels": (_i64, [_vp]),
    "esim_plan_worklist_capacity": (_i64, [_vp]),
    "esim_plan_pixel_offset": (_i64, [_vp, _i32]),
    "esim_plan_set_schedule": (_i32, [_vp, _i32, _i32, _i32]),
    "esim_log_brightness": (_i32, [_vp, _vp, _i64, _f32, _vp]),
    "esim_wlr_threshold": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "esim_wlr_regress": (_i32, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "esim_events": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp]),
    "esim_step": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "esim_backward_scratch_bytes": (_sz, [_vp, _i64]),
    "esim_wlr_backward": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "esim_log_variance": (_i32, [_vp, _vp, _i32, _vp, _i64, _f32, _vp]),
    "esim_wlr_regress_bandwidth": (_i32, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _i32, _vp, _vp, _vp, _vp,
                                          _vp]),
    "esim_nn_scratch_bytes": (_sz, [_i32, _i32, _i32]),
    "esim_nn_distances": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 _vp, _vp, _sz, _vp]),
    "esim_nn_distances_noalloc": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         _vp, _vp]),
    "esim_status_string": (ctypes.c_char_p, [_i32]),
    "esim_last_error": (ctypes.c_char_p, []),
    "esim_build_info": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libesim.so (built by ``paper_2303_02608_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libesim.so is not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != OK:
        msg = load().esim_last_error().decode()
        raise EsimError(status, where, msg)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        if not torch.cuda.is_available():
            return None
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


class Params:
    """Method parameters of one clip (mirrors esim_params)."""

    def __init__(self, r: int, tr: int, C: float, h: float = 1.0,
                 b: Optional[Sequence[float]] = None, ridge: float = 1e-6,
                 precision: int = GRAM_F64, kappa_fp64: float = 1e6, multi_crossing: bool = False,
                 threshold: int = THRESHOLD_CLOSED, dt: float = 1.0):
        self.r, self.tr, self.C, self.h = int(r), int(tr), float(C), float(h)
        self.b = None if b is None else [float(v) for v in b]
        self.ridge, self.precision, self.kappa_fp64 = float(ridge), int(precision), float(kappa_fp64)
        self.multi_crossing = bool(multi_crossing)
        self.threshold = int(threshold)
        self.dt = float(dt)

    def struct(self, F: int) -> esim_params:
        b = [1.0] * (F + 2) if self.b is None else list(self.b)
        if len(b) != F + 2:
            raise ValueError(f"b needs F+2 = {F + 2} values")
        arr = (ctypes.c_double * MAX_D)(*(b + [1.0] * (MAX_D - len(b))))
        return esim_params(self.r, self.tr, self.C, self.h, arr, self.ridge, self.precision,
                           self.kappa_fp64, int(self.multi_crossing), self.threshold, self.dt)


class State:
    """Per-pixel reference state of one clip (device tensors)."""

    def __init__(self, H: int, W: int, F: int, device):
        HW = H * W
        self.alpha = torch.zeros(HW, dtype=torch.float32, device=device)
        self.beta = torch.zeros((F, HW), dtype=torch.float32, device=device)
        self.xref = torch.zeros((F, HW), dtype=torch.float32, device=device)
        self.tref = torch.zeros(HW, dtype=torch.int32, device=device)
        self.last = torch.zeros(HW, dtype=torch.float32, device=device)
        self.bxy = torch.zeros((2, HW), dtype=torch.float32, device=device)
        self.rmom = torch.zeros((2, HW), dtype=torch.float32, device=device)

    def struct(self) -> esim_state:
        return esim_state(_ptr(self.alpha), _ptr(self.beta), _ptr(self.xref), _ptr(self.tref),
                          _ptr(self.last), _ptr(self.bxy), _ptr(self.rmom))


class Plan:
    """A set of clips with their parameters and states (esim_plan)."""

    def __init__(self, ys: List[torch.Tensor], feats: List[torch.Tensor],
                 params: List[Params], states: Optional[List[State]] = None):
        lib = load()
        n = len(ys)
        assert n == len(feats) == len(params) and n >= 1
        self.ys, self.feats, self.params = ys, feats, params
        self.states = states if states is not None else [
            State(f.shape[2], f.shape[3], f.shape[1], f.device) for f in feats]
        clips = (esim_clip * n)()
        pars = (esim_params * n)()
        sts = (esim_state * n)()
        for i, (y, f, p, s) in enumerate(zip(ys, feats, params, self.states)):
            T, F, H, W = f.shape
            if y.shape != (T, H, W) or y.dtype != torch.float32 or not y.is_contiguous():
                raise ValueError("y must be contiguous float32 [T][H][W]")
            if f.dtype not in (torch.float32, torch.float16) or not f.is_contiguous():
                raise ValueError("feat must be contiguous float32/float16 [T][F][H][W]")
            clips[i] = esim_clip(W, H, T, F, F16 if f.dtype == torch.float16 else F32,
                                 _ptr(y), _ptr(f))
            pars[i] = p.struct(F)
            sts[i] = s.struct()
        h = ctypes.c_void_p()
        _check(lib.esim_plan_create(ctypes.addressof(clips), ctypes.addressof(pars),
                                    ctypes.addressof(sts), n, ctypes.byref(h)), "plan_create")
        self.h = h
        self.npix = lib.esim_plan_pixels(h)
        self.wl_capacity = lib.esim_plan_worklist_capacity(h)
        self.offsets = [lib.esim_plan_pixel_offset(h, i) for i in range(n)]
        self.F = feats[0].shape[1]
        self.D = self.F + 2
        self.schedule = (4, 16, 4)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.esim_plan_destroy(h)
            self.h = None

    def set_schedule(self, lanes_dense: int, lanes_list: int, blocks_per_cu: int):
        _check(load().esim_plan_set_schedule(self.h, lanes_dense, lanes_list, blocks_per_cu),
               "set_schedule")
        self.schedule = (lanes_dense, lanes_list, blocks_per_cu)


class Events:
    """Device event buffers (SoA) with a running count."""

    def __init__(self, capacity: int, device, with_clip: bool = False, with_ts: bool = False):
        self.capacity = int(capacity)
        self.x = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.y = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.t = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.p = torch.empty(self.capacity, dtype=torch.int8, device=device)
        self.clip = torch.empty(self.capacity, dtype=torch.int32, device=device) if with_clip else None
        self.ts = torch.empty(self.capacity, dtype=torch.float32, device=device) if with_ts else None
        self.count = torch.zeros(1, dtype=torch.int64, device=device)

    def struct(self) -> esim_events_buf:
        return esim_events_buf(_ptr(self.x), _ptr(self.y), _ptr(self.t), _ptr(self.p),
                               _ptr(self.clip), self.capacity, _ptr(self.count), _ptr(self.ts))

    def host(self):
        n = int(self.count.item())
        m = min(n, self.capacity)
        out = dict(x=self.x[:m].cpu().numpy(), y=self.y[:m].cpu().numpy(),
                   t=self.t[:m].cpu().numpy(), p=self.p[:m].cpu().numpy(), count=n)
        if self.clip is not None:
            out["clip"] = self.clip[:m].cpu().numpy()
        if self.ts is not None:
            out["ts"] = self.ts[:m].cpu().numpy()
        return out


# ---------------------------------------------------------------------------
# thin wrappers of the entry points
# ---------------------------------------------------------------------------
def log_brightness(E: torch.Tensor, eps: float = 1e-3, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    if E.dtype != torch.float32 or not E.is_contiguous():
        raise ValueError("E must be contiguous float32")
    y = torch.empty_like(E) if out is None else out
    _check(load().esim_log_brightness(_ptr(E), _ptr(y), E.numel(), eps, _stream(stream)),
           "log_brightness")
    return y


def log_variance(E: torch.Tensor, var: torch.Tensor, spp: int, eps: float = 1e-3,
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """MC variance of y = log(E + eps) for the mean E of spp samples with
    sample variance var (esim_log_variance)."""
    for t in (E, var):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("E and var must be contiguous float32")
    if var.shape != E.shape:
        raise ValueError("E and var shapes differ")
    vy = torch.empty_like(E) if out is None else out
    _check(load().esim_log_variance(_ptr(E), _ptr(var), int(spp), _ptr(vy), E.numel(), eps,
                                    _stream(stream)), "log_variance")
    return vy


def regress_bandwidth(plan: Plan, t: int, worklist: Optional[torch.Tensor], count: Optional[torch.Tensor],
                      n_out: int, vy: torch.Tensor, hs: Sequence[float], alpha: torch.Tensor,
                      beta: Optional[torch.Tensor] = None, hsel: Optional[torch.Tensor] = None,
                      sure: Optional[torch.Tensor] = None, stream=None):
    """Bandwidth-optimised regression at frame t (esim_wlr_regress_bandwidth):
    the candidate h of hs with the smallest SURE, per item."""
    arr = (ctypes.c_double * len(hs))(*[float(h) for h in hs])
    _check(load().esim_wlr_regress_bandwidth(plan.h, t, _ptr(worklist), _ptr(count), n_out, _ptr(vy), arr,
                                             len(hs), _ptr(alpha), _ptr(beta), _ptr(hsel), _ptr(sure),
                                             _stream(stream)), "wlr_regress_bandwidth")


def threshold(plan: Plan, t: int, dl: torch.Tensor, worklist: torch.Tensor, count: torch.Tensor,
              stream=None):
    _check(load().esim_wlr_threshold(plan.h, t, _ptr(dl), _ptr(worklist), _ptr(count),
                                     _stream(stream)), "wlr_threshold")


def regress(plan: Plan, t: int, worklist: Optional[torch.Tensor], count: Optional[torch.Tensor],
            n_out: int, alpha: torch.Tensor, beta: Optional[torch.Tensor] = None,
            resid: Optional[torch.Tensor] = None, kappa: Optional[torch.Tensor] = None,
            stream=None):
    _check(load().esim_wlr_regress(plan.h, t, _ptr(worklist), _ptr(count), n_out, _ptr(alpha),
                                   _ptr(beta), _ptr(resid), _ptr(kappa), _stream(stream)),
           "wlr_regress")


def events(plan: Plan, t: int, mode: int, ev: Optional[Events], worklist=None, count=None,
           dl=None, alpha=None, beta=None, n_out: int = 0, stream=None):
    evs = ev.struct() if ev is not None else None
    _check(load().esim_events(plan.h, t, mode, _ptr(worklist), _ptr(count), _ptr(dl), _ptr(alpha),
                              _ptr(beta), n_out, ctypes.byref(evs) if evs is not None else None,
                              _stream(stream)), "events")


def step(plan: Plan, t: int, mode: int, ev: Optional[Events] = None, dl=None, stream=None):
    """One frame of a conversion with the plan's own work buffers (esim_step)."""
    evs = ev.struct() if ev is not None else None
    _check(load().esim_step(plan.h, t, mode, _ptr(dl), ctypes.byref(evs) if evs is not None else None,
                            _stream(stream)), "step")


def nn_distances(src: dict, qry: dict, W: int, H: int, T: int, rmax: float, scales=None,
                 scratch: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Distance from every query event to the nearest source event of the same
    polarity (esim_nn_distances); src/qry: dicts of device tensors x, y, t
    (int32) and p (int8).  Scales default to 1/W, 1/H, 1/T."""
    sx, sy, st = scales if scales is not None else (1.0 / W, 1.0 / H, 1.0 / T)
    nq = int(qry["x"].numel())
    dev = qry["x"].device
    d = torch.empty(nq, dtype=torch.float64, device=dev)
    need = int(load().esim_nn_scratch_bytes(W, H, T))
    if scratch is None or scratch.numel() * scratch.element_size() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(load().esim_nn_distances(_ptr(src["x"]), _ptr(src["y"]), _ptr(src["t"]), _ptr(src["p"]),
                                    int(src["x"].numel()), _ptr(qry["x"]), _ptr(qry["y"]), _ptr(qry["t"]),
                                    _ptr(qry["p"]), nq, W, H, T, sx, sy, st, float(rmax), _ptr(d),
                                    _ptr(scratch), scratch.numel() * scratch.element_size(),
                                    _stream(stream)), "nn_distances")
    return d


NN_STATIC_BYTES = 32 << 20     # ESIM_NN_STATIC_BYTES


def nn_distances_noalloc(src: dict, qry: dict, W: int, H: int, T: int, rmax: float, d: torch.Tensor,
                         scales=None, stream=None) -> torch.Tensor:
    """nn_distances with the library's fixed bitmap array: allocates nothing
    (esim_nn_distances_noalloc); d (float64, one per query) is the output."""
    sx, sy, st = scales if scales is not None else (1.0 / W, 1.0 / H, 1.0 / T)
    nq = int(qry["x"].numel())
    if d.dtype != torch.float64 or d.numel() < nq:
        raise ValueError("d must be float64 with one value per query")
    _check(load().esim_nn_distances_noalloc(_ptr(src["x"]), _ptr(src["y"]), _ptr(src["t"]), _ptr(src["p"]),
                                            int(src["x"].numel()), _ptr(qry["x"]), _ptr(qry["y"]), _ptr(qry["t"]),
                                            _ptr(qry["p"]), nq, W, H, T, sx, sy, st, float(rmax), _ptr(d),
                                            _stream(stream)), "nn_distances_noalloc")
    return d


def backward_scratch_bytes(plan: Plan, n: int) -> int:
    return int(load().esim_backward_scratch_bytes(plan.h, n))


def backward(plan: Plan, items: torch.Tensor, g_alpha: torch.Tensor, g_y: torch.Tensor,
             g_b: torch.Tensor, scratch: torch.Tensor, stream=None):
    _check(load().esim_wlr_backward(plan.h, _ptr(items), items.numel(), _ptr(g_alpha), _ptr(g_y),
                                    _ptr(g_b), _ptr(scratch), scratch.numel() * scratch.element_size(),
                                    _stream(stream)), "wlr_backward")
