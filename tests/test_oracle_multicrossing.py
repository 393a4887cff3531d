"""Pins of the oracle's every-crossing event rule (ESIM proper: eq. 1 of
Sec. 1.1 applied to every level the brightness passes between two frames,
modes RAW_ALL and EXHAUSTIVE_ALL of ``oracle.run``).

What fixes the rule independently of the oracle's code:
- a brightness ramp crosses the levels L_0 + k C at the closed-form times
  k C / s;
- the fixed-step ESIM of eq. 1 (fire when |L - L_ref| >= C, then L_ref <- L)
  run on the frames linearly interpolated at a fine time step converges to
  the every-crossing rule as the step shrinks: same events, times within the
  step;
- invariants: after each frame |L_t - L_ref| < C and L_ref stays on the
  lattice L_0 + C Z; per pixel the times increase and lie in (t - 1, t];
- symmetries: y + c changes nothing, -y flips every polarity;
- the exhaustive form is the raw form applied to the oracle's own regressed
  alpha, and equals the raw form when the feature weights underflow (h -> 0).
"""
import numpy as np
import pytest

import oracle


def _clip_from_y(y):
    """A clip whose brightness is y [T][H][W] (features unused by the raw rule)."""
    T, H, W = y.shape
    return oracle.Clip(np.asarray(y, np.float64), np.zeros((T, 1, H, W), np.float32))


def _raw_all(y, C):
    clip = _clip_from_y(y)
    return oracle.run(clip, oracle.Params(r=1, tr=0, C=C), oracle.RAW_ALL, want_dl=True)


def test_ramp_closed_form():
    C, s, L0 = 0.25, 0.6 + 1e-3 * np.sqrt(2.0), -1.0      # about 2.4 C per frame
    T = 7
    y = (L0 + s * np.arange(T, dtype=np.float64))[:, None, None]
    o = _raw_all(y, C)
    ex, ey, et, ep = o["events"]
    kmax = int(np.floor(s * (T - 1) / C))
    assert o["count"] == kmax
    k = np.arange(1, kmax + 1)
    t_cross = k * C / s
    assert np.all(ep == 1)
    assert np.allclose(o["ts"], t_cross, rtol=0, atol=1e-12)
    assert np.array_equal(et, np.ceil(t_cross).astype(np.int32))
    # the final reference is the last level passed, not the last value
    assert o["state"]["alpha"][0] == pytest.approx(L0 + kmax * C, abs=1e-12)


def test_fine_step_esim_converges_to_every_crossing():
    rng = np.random.default_rng(3)
    T, n, C = 6, 5, 0.3
    y = np.cumsum(rng.normal(0.0, 0.5, (T, 1, n)), axis=0)
    o = _raw_all(y, C)
    ex, ey, et, ep = o["events"]
    M = 20000                                          # sub-steps per frame
    for q in range(n):
        L = y[:, 0, q]
        tau = np.arange((T - 1) * M + 1) / M
        Lf = np.interp(tau, np.arange(T), L)
        ref = L[0]
        times, pols = [], []
        for i in range(1, tau.size):
            d = Lf[i] - ref
            if abs(d) >= C:                              # eq. 1 at the fine step
                times.append(tau[i])
                pols.append(1 if d > 0 else -1)
                ref = Lf[i]
        m = ex == q
        assert m.sum() == len(times), q
        assert np.array_equal(ep[m], np.array(pols, np.int8))
        # each fine-step event lies within a step after the crossing, plus the
        # time the signal takes to cover the reference's drift (each fine-step
        # event overshoots its level by at most one step's change)
        smax = np.max(np.abs(np.diff(L)))
        local = np.abs(np.diff(L))[et[m] - 1]
        drift = np.arange(1, len(times) + 1) * smax / M
        tol = 1.0 / M + drift / local + 1e-12
        assert np.all(np.abs(o["ts"][m] - np.array(times)) <= tol)


def test_invariants_on_random_walks():
    rng = np.random.default_rng(5)
    T, H, W, C = 9, 3, 4, 0.2
    y = np.cumsum(rng.normal(0.0, 0.45, (T, H, W)), axis=0)
    o = _raw_all(y, C)
    ex, ey, et, ep = o["events"]
    pix = ey.astype(np.int64) * W + ex
    L0 = y[0].reshape(-1)
    for t in range(1, T):
        # the state after frame t, from a run over frames 0..t
        ref = _raw_all(y[: t + 1], C)["state"]["alpha"]
        Lt = y[t].reshape(-1)
        assert np.all(np.abs(Lt - ref) < C)
        m = et <= t
        net = np.bincount(pix[m], weights=ep[m].astype(np.float64), minlength=H * W)
        assert np.allclose(ref - L0, C * net, rtol=0, atol=1e-12)
        # the count of frame t is floor(|L_t - L_ref before t| / C)
        prev = _raw_all(y[:t], C)["state"]["alpha"]
        cnt = np.bincount(pix[et == t], minlength=H * W)
        assert np.array_equal(cnt, np.floor(np.abs(Lt - prev) / C).astype(np.int64))
    for q in range(H * W):
        m = pix == q
        assert np.all(np.diff(o["ts"][m]) > 0)
        assert np.all((o["ts"][m] > et[m] - 1) & (o["ts"][m] <= et[m]))


def test_reversal_and_below_threshold():
    C = 0.5
    y = np.array([0.0, 1.2, 1.4, 0.1, 0.2])[:, None, None]
    o = _raw_all(y, C)
    ex, ey, et, ep = o["events"]
    # 0 -> 1.2: levels 0.5, 1.0 (ref 1.0); 1.4: none; 0.1: d = -0.9, one at
    # 0.5 (ref 0.5); 0.2: d = -0.3, none
    assert list(et) == [1, 1, 3]
    assert list(ep) == [1, 1, -1]
    assert o["ts"] == pytest.approx([0.5 / 1.2, 1.0 / 1.2, 2 + (1.4 - 0.5) / 1.3], abs=1e-12)
    # nothing below C, nothing for a constant signal
    assert _raw_all(0.1 * y, C)["count"] == 0
    assert _raw_all(np.ones((5, 2, 2)), C)["count"] == 0


def test_symmetries():
    rng = np.random.default_rng(7)
    y = np.cumsum(rng.normal(0.0, 0.4, (8, 3, 3)), axis=0)
    C = 0.25
    a = _raw_all(y, C)
    b = _raw_all(y + 3.0, C)
    c = _raw_all(-y, C)
    for k in range(3):
        assert np.array_equal(a["events"][k], b["events"][k])
        assert np.array_equal(a["events"][k], c["events"][k])
    assert np.array_equal(a["events"][3], b["events"][3])
    assert np.array_equal(a["events"][3], -c["events"][3])
    assert np.allclose(a["ts"], b["ts"], atol=1e-9) and np.allclose(a["ts"], c["ts"], atol=1e-12)


def test_exhaustive_is_raw_rule_on_alpha(small_clip):
    """Mode EXHAUSTIVE_ALL is the raw every-crossing rule applied to the
    oracle's regressed alpha of every pixel-frame (Sec. 3: ESIM after WLR)."""
    E, feat = small_clip["E"][:6], small_clip["feat"][:6]
    T, F, H, W = feat.shape
    p = oracle.Params(r=3, tr=0, C=0.05)
    clip = oracle.Clip(oracle.log_brightness(E), feat)
    ex = oracle.run(clip, p, oracle.EXHAUSTIVE_ALL)
    items = np.arange(T * H * W, dtype=np.int64)
    alpha = oracle.regress_items(clip, p, items)["theta"][:, 0].reshape(T, H, W)
    raw = _raw_all(alpha, p.C)
    assert ex["count"] == raw["count"] > H * W
    for k in range(4):
        assert np.array_equal(ex["events"][k], raw["events"][k])
    assert np.allclose(ex["ts"], raw["ts"], rtol=0, atol=1e-12)


def test_exhaustive_equals_raw_when_weights_underflow(small_clip):
    """h -> 0: every neighbour's weight underflows, alpha = y at the centre
    (the ridge keeps the system solvable), so both every-crossing forms agree."""
    E, feat = small_clip["E"][:5], small_clip["feat"][:5]
    clip = oracle.Clip(oracle.log_brightness(E), feat)
    p = oracle.Params(r=2, tr=0, C=0.1, h=1e-6, ridge=1e-3)
    a = oracle.run(clip, p, oracle.EXHAUSTIVE_ALL)
    b = oracle.run(clip, p, oracle.RAW_ALL)
    assert a["count"] == b["count"] > 0
    for k in range(4):
        assert np.array_equal(a["events"][k], b["events"][k])
    assert np.allclose(a["ts"], b["ts"], rtol=0, atol=1e-9)
