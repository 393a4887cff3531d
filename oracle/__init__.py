"""FP64 CPU oracle of the event simulator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
binding) never touches it, and it shares no code with them.

The arithmetic lives in ``esim_oracle.cpp`` (plain C++, double precision); this
module loads it with ctypes and marshals numpy arrays.  Every function cites
the passage of the paper it follows (Tsuji et al., arXiv 2303.02608).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esim_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

THRESHOLDED, EXHAUSTIVE, RAW = 0, 1, 2
# thresholded with Delta R = |R_hat - R| evaluated explicitly (eqs. 4 and 7):
# R_hat over the last-event window, or over the current frame's window
EXPLICIT_LAST, EXPLICIT_NEW = 3, 4
# WLR+ESIM and ESIM with every crossing (eq. 1 applied to each level passed
# between two frames, at interpolated times)
EXHAUSTIVE_ALL, RAW_ALL = 5, 6


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Clip(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("T", ctypes.c_int32),
                ("F", ctypes.c_int32), ("y", ctypes.c_void_p), ("feat", ctypes.c_void_p),
                ("feat_f16", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("tr", ctypes.c_int32), ("C", ctypes.c_double),
                ("h", ctypes.c_double), ("b", ctypes.c_void_p), ("ridge", ctypes.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        _lib.orc_log_brightness.argtypes = [vp, vp, i64, dbl]
        _lib.orc_regress.argtypes = [vp, vp, i32, i32, i32, vp, vp, i32]
        _lib.orc_regress.restype = i32
        _lib.orc_normal_equations.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
        _lib.orc_normal_equations.restype = i32
        _lib.orc_window.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, i32]
        _lib.orc_window.restype = i32
        _lib.orc_regress_items.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, i32]
        _lib.orc_regress_items.restype = i32
        _lib.orc_residual_hat.argtypes = [vp, vp, i32, i32, i32, vp, vp]
        _lib.orc_residual_hat.restype = dbl
        _lib.orc_explicit.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
        _lib.orc_explicit.restype = i32
        _lib.orc_log_variance.argtypes = [vp, vp, i32, vp, i64, dbl]
        _lib.orc_regress_bandwidth.argtypes = [vp, vp, vp, i32, vp, vp, i64, vp, vp, vp, vp, i32]
        _lib.orc_regress_bandwidth.restype = i32
        _lib.orc_cond.argtypes = [vp, i32]
        _lib.orc_cond.restype = dbl
        _lib.orc_run.argtypes = [vp, vp, i32, vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp,
                                 vp, vp, i32, vp, i32, vp]
        _lib.orc_run.restype = i64
        _lib.orc_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        _lib.orc_backward.restype = i32
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


@dataclass
class Params:
    """Method parameters: radius r, temporal radius tr (frames), contrast
    threshold C, bandwidths h and b[F+2] (coordinates first), ridge lambda on
    the beta block."""
    r: int
    tr: int
    C: float
    h: float = 1.0
    b: Optional[Sequence[float]] = None
    ridge: float = 1e-6


class Clip:
    """A clip as the oracle sees it: y[T][H][W] (double, log brightness) and
    feat[T][F][H][W] (float32 or float16)."""

    def __init__(self, y: np.ndarray, feat: np.ndarray):
        y = np.ascontiguousarray(y, dtype=np.float64)
        if feat.dtype not in (np.float32, np.float16):
            feat = feat.astype(np.float32)
        feat = np.ascontiguousarray(feat)
        T, F, H, W = feat.shape
        assert y.shape == (T, H, W), (y.shape, feat.shape)
        self.y, self.feat = y, feat
        self.T, self.F, self.H, self.W = T, F, H, W
        self._c = _Clip(W, H, T, F, y.ctypes.data, feat.ctypes.data,
                        1 if feat.dtype == np.float16 else 0)

    @property
    def D(self):
        return self.F + 2

    @property
    def P(self):
        return self.F + 3


def _params(clip: Clip, p: Params):
    b = np.ones(clip.D) if p.b is None else np.asarray(p.b, dtype=np.float64)
    assert b.shape == (clip.D,)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return _Params(p.r, p.tr, p.C, p.h, b.ctypes.data, p.ridge), b


def log_brightness(E: np.ndarray, eps: float = 1e-3) -> np.ndarray:
    """Sec. 1.1 / Sec. 2.1: y := L = log E, with eps inside the log."""
    E = np.ascontiguousarray(E, dtype=np.float32)
    y = np.empty(E.shape, dtype=np.float64)
    _L().orc_log_brightness(E.ctypes.data, y.ctypes.data, E.size, eps)
    return y


def regress(clip: Clip, p: Params, t: int, px: int, py: int, kappa: bool = False):
    """Eqs. (3)-(5): one weighted local regression.  Returns (theta, info) with
    theta = (alpha, beta_x, beta_y, beta_f...) and info = dict(W, R, kappa, ok)."""
    cp, b = _params(clip, p)
    theta = np.empty(clip.P)
    info = np.empty(4)
    _L().orc_regress(ctypes.byref(clip._c), ctypes.byref(cp), t, px, py, theta.ctypes.data,
                     info.ctypes.data, 1 if kappa else 0)
    return theta, dict(W=info[0], R=info[1], kappa=info[2], ok=bool(info[3]))


def normal_equations(clip: Clip, p: Params, t: int, px: int, py: int):
    """The W-normalised Gram (with ridge), right-hand side and W of eq. (4)."""
    cp, b = _params(clip, p)
    A = np.empty((clip.P, clip.P))
    g = np.empty(clip.P)
    W = np.empty(1)
    n = _L().orc_normal_equations(ctypes.byref(clip._c), ctypes.byref(cp), t, px, py,
                                  A.ctypes.data, g.ctypes.data, W.ctypes.data)
    return A, g, float(W[0]), n


def window(clip: Clip, p: Params, t: int, px: int, py: int):
    """The window samples of eq. (5): positions (t, py, px), weights w, z=(1,u)."""
    cp, b = _params(clip, p)
    cap = (2 * p.r + 1) ** 2 * (2 * p.tr + 1)
    pos = np.empty((cap, 3), dtype=np.int32)
    w = np.empty(cap)
    z = np.empty((cap, clip.P))
    n = _L().orc_window(ctypes.byref(clip._c), ctypes.byref(cp), t, px, py, pos.ctypes.data,
                        w.ctypes.data, z.ctypes.data, cap)
    return pos[:n], w[:n], z[:n]


def regress_items(clip: Clip, p: Params, items: np.ndarray, kappa: bool = False,
                  nthreads: int = 0):
    """Regressions at items = t*H*W + py*W + px.  Returns dict(theta[n][P], W, R,
    kappa, fails)."""
    cp, b = _params(clip, p)
    items = np.ascontiguousarray(items, dtype=np.int64)
    n = items.size
    theta = np.empty((n, clip.P))
    W = np.empty(n)
    R = np.empty(n)
    K = np.empty(n) if kappa else None
    fails = _L().orc_regress_items(ctypes.byref(clip._c), ctypes.byref(cp), items.ctypes.data,
                                   n, theta.ctypes.data, W.ctypes.data, R.ctypes.data, _p(K),
                                   nthreads)
    return dict(theta=theta, W=W, R=R, kappa=K, fails=fails)


def residual_hat(clip: Clip, p: Params, t_ref: int, px: int, py: int, xhat: np.ndarray):
    """Eq. (7) evaluated explicitly over the last-event window.  Returns (R_hat, R)."""
    cp, b = _params(clip, p)
    xhat = np.ascontiguousarray(xhat, dtype=np.float64)
    R = np.empty(1)
    Rh = _L().orc_residual_hat(ctypes.byref(clip._c), ctypes.byref(cp), t_ref, px, py,
                               xhat.ctypes.data, R.ctypes.data)
    return float(Rh), float(R[0])


def explicit(clip: Clip, p: Params, new_window: bool, t_ref: int, t: int, px: int, py: int,
             theta: np.ndarray):
    """Delta R of Sec. 2.2 evaluated explicitly for the plane theta = (alpha,
    beta over D) regressed at (t_ref, py, px): R (eq. 4) over the plane's own
    window and R_hat (eq. 7) over the last-event window, or (new_window) over
    frame t's window centred at frame t's feature vector.  Returns dict(R,
    R_hat, mean, change): mean is the weighted mean of the translated plane's
    residuals, change = sign(mean) * sqrt(|R_hat - R|)."""
    cp, b = _params(clip, p)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    assert theta.size == clip.P
    out = np.empty(4)
    rc = _L().orc_explicit(ctypes.byref(clip._c), ctypes.byref(cp), 1 if new_window else 0, t_ref, t,
                           px, py, theta.ctypes.data, out.ctypes.data)
    assert rc == 0, rc
    return dict(R=float(out[0]), R_hat=float(out[1]), mean=float(out[2]), change=float(out[3]))


def log_variance(E: np.ndarray, var: np.ndarray, spp: int, eps: float = 1e-3) -> np.ndarray:
    """Variance of y = log(E + eps) for the mean E of spp samples whose unbiased
    sample variance is var (delta method): var / spp / (E + eps)^2."""
    E = np.ascontiguousarray(E, dtype=np.float32)
    var = np.ascontiguousarray(var, dtype=np.float32)
    vy = np.empty(E.shape, np.float64)
    _L().orc_log_variance(E.ctypes.data, var.ctypes.data, int(spp), vy.ctypes.data, E.size, eps)
    return vy


def regress_bandwidth(clip: Clip, p: Params, hs, vy: np.ndarray, items: np.ndarray,
                      nthreads: int = 0):
    """The bandwidth-optimised regression (Sec. 3, bandwidth optimisation; the
    estimator is a reading): for each item (t*H*W + pixel) the candidate global
    bandwidth h of eq. (5) with the smallest SURE_k = (alpha_k - y_c)^2 +
    2 vy_c v_0 / W_k - vy_c, v = A^{-1} e_0.  Returns dict(theta [n][P], h [n],
    alpha_k [n][K], sure [n][K], fails)."""
    cp, b = _params(clip, p)
    hs = np.ascontiguousarray(hs, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    assert vy.shape == (clip.T, clip.H, clip.W)
    items = np.ascontiguousarray(items, dtype=np.int64)
    n, K = items.size, hs.size
    theta = np.empty((n, clip.P))
    h = np.empty(n)
    ak = np.empty((n, K))
    sk = np.empty((n, K))
    fails = _L().orc_regress_bandwidth(ctypes.byref(clip._c), ctypes.byref(cp), hs.ctypes.data, K,
                                       vy.ctypes.data, items.ctypes.data, n, theta.ctypes.data,
                                       h.ctypes.data, ak.ctypes.data, sk.ctypes.data, nthreads)
    return dict(theta=theta, h=h, alpha_k=ak, sure=sk, fails=fails)


def cond(A: np.ndarray) -> float:
    """2-norm condition number of a symmetric positive definite matrix (Jacobi)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    return float(_L().orc_cond(A.ctypes.data, A.shape[0]))


def run(clip: Clip, p: Params, mode: int = THRESHOLDED, pixels: Optional[np.ndarray] = None,
        want_dl: bool = False, check_identity: bool = False, cap: Optional[int] = None,
        nthreads: int = 0):
    """Event simulation (Sec. 1.1 eq. 1; Sec. 2.2 Prop. 1; Sec. 3 baselines;
    EXPLICIT_LAST / EXPLICIT_NEW: Sec. 2.2 with Delta R evaluated explicitly,
    dl then holding sign * sqrt(Delta R); EXHAUSTIVE_ALL / RAW_ALL: the
    baselines with every crossing, ESIM proper).

    Returns dict(events=(x, y, t, p) int arrays in (t, py, px) order (the
    crossings of one pixel-frame in time order), ts = event times in frame
    units (the interpolated crossing times in the every-crossing modes), count,
    dl [T][npix] (if asked), nflag[T], state (alpha, beta[F][npix], xref,
    tref), identity_err)."""
    cp, b = _params(clip, p)
    HW = clip.H * clip.W
    if pixels is not None:
        pixels = np.ascontiguousarray(np.sort(np.asarray(pixels, dtype=np.int32)))
        npix = pixels.size
    else:
        npix = HW
    if cap is None:
        cap = max(16, npix * clip.T)
    while True:
        ex = np.empty(cap, np.int32)
        ey = np.empty(cap, np.int32)
        et = np.empty(cap, np.int32)
        ep = np.empty(cap, np.int8)
        ets = np.empty(cap, np.float64)
        dl = np.empty((clip.T, npix)) if want_dl else None
        nflag = np.empty(clip.T, np.int64)
        st_a = np.empty(npix)
        st_b = np.empty((clip.F, npix))
        st_x = np.empty((clip.F, npix))
        st_t = np.empty(npix, np.int32)
        err = np.zeros(1)
        n = _L().orc_run(ctypes.byref(clip._c), ctypes.byref(cp), mode, _p(pixels), npix,
                         ex.ctypes.data, ey.ctypes.data, et.ctypes.data, ep.ctypes.data, cap,
                         _p(dl), nflag.ctypes.data, st_a.ctypes.data, st_b.ctypes.data,
                         st_x.ctypes.data, st_t.ctypes.data, 1 if check_identity else 0,
                         err.ctypes.data, nthreads, ets.ctypes.data)
        if n <= cap or mode not in (EXHAUSTIVE_ALL, RAW_ALL):
            break
        cap = int(n)        # several events per pixel-frame: run again with room for all
    m = min(n, cap)
    return dict(events=(ex[:m].copy(), ey[:m].copy(), et[:m].copy(), ep[:m].copy()), count=int(n),
                ts=ets[:m].copy(), dl=dl, nflag=nflag,
                state=dict(alpha=st_a, beta=st_b, xref=st_x, tref=st_t),
                identity_err=float(err[0]), pixels=pixels)


def backward(clip: Clip, p: Params, items: np.ndarray, galpha: np.ndarray):
    """Adjoint of alpha at items (t*H*W + pixel) under upstream gradients
    galpha.  Returns (g_y [T][H][W], g_b [F+2], fails)."""
    cp, b = _params(clip, p)
    items = np.ascontiguousarray(items, dtype=np.int64)
    galpha = np.ascontiguousarray(galpha, dtype=np.float64)
    gy = np.zeros((clip.T, clip.H, clip.W))
    gb = np.zeros(clip.D)
    fails = _L().orc_backward(ctypes.byref(clip._c), ctypes.byref(cp), items.ctypes.data,
                              items.size, galpha.ctypes.data, gy.ctypes.data, gb.ctypes.data)
    return gy, gb, fails
