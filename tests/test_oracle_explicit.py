"""Pins of the explicit thresholds of the oracle (Sec. 2.2, eqs. 4 and 7
evaluated from their definitions rather than through Prop. 1).

  - Over the last-event window, R_hat - R equals the closed form's dL^2 at the
    least-squares minimiser (the alpha normal equation makes the residuals'
    weighted mean zero): the explicit run equals the closed-form run.
  - Over the current frame's window, a brightness change that the features do
    not explain (y_t = y_0 + delta_t, features static, single-frame windows)
    gives translated residuals r_i + delta, so R_hat - R = delta^2 and the mean
    is delta: the events are eq. (1) applied to delta_t at every pixel, while
    both last-window forms see nothing (the limitation of a threshold driven by
    features only).
  - A noise-free affine scene (ridge 0) is fitted exactly, so over the current
    window every translated residual equals dL: all three forms agree.
  - Brute force on one tiny window, written out here with numpy loops.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2303_02608_amd import synth


def _clip_from(y, feat):
    return oracle.Clip(np.asarray(y, np.float64), np.asarray(feat, np.float32))


def _events(out):
    x, y, t, p = out["events"]
    return [(int(a), int(b), int(c), int(d)) for a, b, c, d in zip(t, y, x, p)]


def _eq1_events(L, C):
    T, H, W = L.shape
    ref = L[0].copy()
    ev = []
    for t in range(1, T):
        d = L[t] - ref
        fire = np.abs(d) >= C
        for py, px in zip(*np.nonzero(fire)):
            ev.append((t, int(py), int(px), 1 if d[py, px] > 0 else -1))
        ref[fire] = L[t][fire]
    return ev


@pytest.mark.parametrize("ridge", [0.0, 1e-3])
def test_last_window_equals_closed_form(small_clip, ridge):
    """R_hat over the last-event window: Delta R = dL^2 and the sign of the
    mean residual is the sign of dL, so the run is the closed-form run."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    T = 6
    clip = oracle.Clip(oracle.log_brightness(E[:T]), feat[:T])
    p = oracle.Params(cfg["r"], 1, cfg["C"], ridge=ridge)
    pix = np.arange(0, 64 * 64, 7)
    a = oracle.run(clip, p, oracle.THRESHOLDED, pixels=pix, want_dl=True)
    b = oracle.run(clip, p, oracle.EXPLICIT_LAST, pixels=pix, want_dl=True)
    da, db = a["dl"][1:], b["dl"][1:]
    # squares agree to rounding (sqrt would magnify rounding near zero)
    assert np.max(np.abs(da * da - db * db)) <= 1e-10
    big = np.abs(da) > 1e-4
    assert np.array_equal(np.sign(da[big]), np.sign(db[big]))
    assert np.nanmin(np.abs(np.abs(da) - p.C)) > 1e-8      # no knife-edge decision
    assert _events(a) == _events(b) and a["count"] > 10


def _flicker_scene(T=12, H=8, W=9, F=3, seed=71):
    d = synth.random_features_clip(W, H, 1, F, seed)
    feat = np.repeat(d["feat"].numpy(), T, axis=0)
    rng = np.random.default_rng(seed)
    y0 = rng.normal(-1.0, 0.3, size=(H, W))
    # global offsets, kept away from the knife edge of C = 0.2
    delta = np.array([0.0, 0.05, 0.13, 0.26, 0.31, 0.12, 0.02, -0.11, -0.35, -0.3, 0.0, 0.07])[:T]
    y = y0[None] + delta[:, None, None]
    return y, feat, delta


@pytest.mark.parametrize("ridge", [0.0, 1e-2])
def test_new_window_sees_brightness_the_features_do_not_explain(ridge):
    y, feat, delta = _flicker_scene()
    T, H, W = y.shape
    C = 0.2
    clip = _clip_from(y, feat)
    p = oracle.Params(r=2, tr=0, C=C, ridge=ridge)
    out = oracle.run(clip, p, oracle.EXPLICIT_NEW, want_dl=True)
    # eq. (1) on delta_t at every pixel
    ref = _eq1_events(np.broadcast_to(delta[:, None, None], (T, H, W)).copy(), C)
    assert _events(out) == ref and len(ref) > 0
    # the compared change is delta_t - delta_ref exactly (up to rounding)
    Lref = delta[0]
    for t in range(1, T):
        d = delta[t] - Lref
        assert np.max(np.abs(out["dl"][t] - d)) <= 1e-9, t
        if abs(d) >= C:
            Lref = delta[t]
    for mode in (oracle.THRESHOLDED, oracle.EXPLICIT_LAST):
        o = oracle.run(clip, p, mode, want_dl=True)
        assert o["count"] == 0, mode
        assert np.nanmax(np.abs(o["dl"])) <= 1e-6


def test_static_clip_gives_no_events_in_any_reading():
    T, F, H, W = 5, 2, 7, 8
    d = synth.random_features_clip(W, H, 1, F, seed=81)
    feat = np.repeat(d["feat"].numpy(), T, axis=0)
    rng = np.random.default_rng(81)
    y = np.repeat(rng.normal(-1.0, 0.4, size=(1, H, W)), T, axis=0)
    clip = _clip_from(y, feat)
    for tr in (0, 1):
        p = oracle.Params(r=2, tr=tr, C=0.05)
        for mode in (oracle.EXPLICIT_LAST, oracle.EXPLICIT_NEW):
            o = oracle.run(clip, p, mode, want_dl=True)
            assert o["count"] == 0
            assert np.nanmax(np.abs(o["dl"])) <= 1e-6


def test_affine_scene_all_readings_agree():
    """Noise-free y = 0.2 + g^T f with moving features, ridge 0: the fit is
    exact, so every translated residual over the current window is dL."""
    T, H, W, F = 14, 10, 12, 3
    d = synth.random_features_clip(W, H, 1, F, 41)
    f0 = d["feat"].numpy()[0].astype(np.float64)
    rng = np.random.default_rng(41)
    vel = rng.uniform(-0.05, 0.05, size=(F, H, W))
    feat = np.stack([f0 + t * vel for t in range(T)]).astype(np.float32)
    g = rng.uniform(-2, 2, size=F)
    y = 0.2 + np.einsum("f,tfhw->thw", g, feat.astype(np.float64))
    clip = _clip_from(y, feat)
    p = oracle.Params(r=2, tr=1, C=0.15, ridge=0.0)
    outs = {m: oracle.run(clip, p, m, want_dl=True)
            for m in (oracle.THRESHOLDED, oracle.EXPLICIT_LAST, oracle.EXPLICIT_NEW)}
    base = outs[oracle.THRESHOLDED]
    assert np.nanmin(np.abs(np.abs(base["dl"][1:]) - p.C)) > 1e-6
    for m, o in outs.items():
        assert _events(o) == _events(base), m
        assert np.nanmax(np.abs(o["dl"][1:] - base["dl"][1:])) <= 1e-6, m
    assert base["count"] > 20


def _brute(y, feat, r, tr, t_ref, t, px, py, theta, new_window):
    """R and R_hat written out with loops: window |dx|,|dy| <= r, |dt| <= tr
    (truncated), x = (px/r, py/r, f), w = exp(-|x - centre|^2 / 2)."""
    T, F, H, W = feat.shape

    def fv(tt, yy, xx):
        return np.concatenate([[xx / r, yy / r], feat[tt, :, yy, xx].astype(np.float64)])

    def window(tt, centre):
        out = []
        for a in range(tt - tr, tt + tr + 1):
            for b in range(py - r, py + r + 1):
                for c in range(px - r, px + r + 1):
                    if 0 <= a < T and 0 <= b < H and 0 <= c < W:
                        x = fv(a, b, c)
                        out.append((math.exp(-0.5 * float(np.sum((x - centre) ** 2))), y[a, b, c], x))
        return out

    xc, xh = fv(t_ref, py, px), fv(t, py, px)
    alpha, beta = theta[0], theta[1:]
    last = window(t_ref, xc)
    Wl = sum(w for w, _, _ in last)
    R = sum(w * (yv - alpha - beta @ (x - xc)) ** 2 for w, yv, x in last) / Wl
    win = window(t, xh) if new_window else last
    Wn = sum(w for w, _, _ in win)
    Rh = sum(w * (yv - alpha - beta @ (x - xh)) ** 2 for w, yv, x in win) / Wn
    m = sum(w * (yv - alpha - beta @ (x - xh)) for w, yv, x in win) / Wn
    return R, Rh, m


@pytest.mark.parametrize("new_window", [False, True])
def test_explicit_matches_brute_force(new_window):
    T, F, H, W = 4, 2, 6, 7
    d = synth.random_features_clip(W, H, T, F, seed=91)
    y = oracle.log_brightness(d["E"].numpy())
    feat = d["feat"].numpy()
    clip = oracle.Clip(y, feat)
    p = oracle.Params(r=2, tr=1, C=0.1)
    for (t_ref, t, px, py) in [(0, 2, 3, 2), (1, 3, 0, 5), (2, 1, 6, 0)]:
        theta, _ = oracle.regress(clip, p, t_ref, px, py)
        got = oracle.explicit(clip, p, new_window, t_ref, t, px, py, theta)
        R, Rh, m = _brute(y, feat, p.r, p.tr, t_ref, t, px, py, theta, new_window)
        assert got["R"] == pytest.approx(R, rel=1e-12, abs=1e-15)
        assert got["R_hat"] == pytest.approx(Rh, rel=1e-12, abs=1e-15)
        assert got["mean"] == pytest.approx(m, rel=1e-12, abs=1e-15)
        assert got["change"] == pytest.approx(math.copysign(math.sqrt(abs(Rh - R)), m if m != 0 else -1.0),
                                              rel=1e-9, abs=1e-12)
