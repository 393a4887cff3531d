"""Explicit Delta R thresholds (Sec. 2.2, eqs. 4 and 7 summed over a window)
on the GPU against the oracle's explicit runs.

Tolerance of the compared change dl = s sqrt(Delta R): the GPU's plane is the
FP32-stored result of its regression (alpha within 1e-4 max(1, |alpha|) of the
oracle's, beta alike), and R, R_hat are quadratic in the plane, so an error
delta in the plane moves Delta R by about 2 (|mean r_hat| + |mean r|) delta +
2 (sigma_r_hat + sigma_r) delta |u|, at most 4 C delta near the threshold, and
dl = sqrt(Delta R) by that over 2 |dl| = 2 C: about 2 delta.  The band is five
times that, 1e-3; as for the closed form, a pixel whose decision differs inside
the band is excused from then on (its states diverge)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from paper_2303_02608_amd.simulator import Simulator
from parity_util import compare_events, oracle_clip, run_gpu, say, to_dev

pytestmark = pytest.mark.gpu

BAND = 1e-3
FORMS = {"last": (B.THRESHOLD_LAST_WINDOW, oracle.EXPLICIT_LAST),
         "new": (B.THRESHOLD_NEW_WINDOW, oracle.EXPLICIT_NEW)}


def _params(cfg, form, **kw):
    return B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], threshold=FORMS[form][0], **kw)


@pytest.mark.parametrize("form", ["last", "new"])
@pytest.mark.parametrize("tr", [0, 1])
def test_explicit_events_match_oracle(small_clip, form, tr):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=tr, C=cfg["C"], threshold=FORMS[form][0])
    say(f"explicit threshold {form} tr={tr} small workload")
    gpu, _ = run_gpu(E, feat, p, "thresholded", keep_dl=True)
    orc = oracle.run(oracle_clip(E, feat), oracle.Params(p.r, p.tr, p.C, p.h, p.b, p.ridge),
                     FORMS[form][1], want_dl=True)
    W = feat.shape[3]
    n, excused, fails = compare_events(gpu, orc, W, p.C, BAND)
    say(f"{form}: gpu {gpu['count']} oracle {orc['count']} events, excused pixels {excused}")
    assert not fails, fails[:10]
    assert excused <= max(2, n // 1000)
    assert gpu["count"] > 0
    g, o = gpu["dl"][1:], orc["dl"][1:]
    both = np.isfinite(g) & np.isfinite(o)
    if excused == 0:
        assert np.max(np.abs(g[both] - o[both])) <= BAND


def test_last_window_equals_closed_form_on_gpu(small_clip):
    """Over the last-event window the explicit sum is the closed form: the
    compared changes agree to the band and the events wherever no decision
    sits inside it."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    say("explicit last window vs closed form")
    a, _ = run_gpu(E, feat, _params(cfg, "last"), "thresholded", keep_dl=True)
    b, _ = run_gpu(E, feat, B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"]), "thresholded", keep_dl=True)
    # the closed-form run as the reference of compare_events (its dl decides the band)
    ref = dict(events=(b["x"], b["y"], b["t"], b["p"]), dl=b["dl"], pixels=None)
    W = feat.shape[3]
    n, excused, fails = compare_events(a, ref, W, cfg["C"], BAND)
    assert not fails, fails[:10]
    assert excused <= max(2, n // 1000)


def _flicker(T=12, H=24, W=40, F=3, seed=71):
    d = synth.random_features_clip(W, H, 1, F, seed)
    feat = np.repeat(d["feat"].numpy(), T, axis=0)
    rng = np.random.default_rng(seed)
    y0 = rng.normal(-1.0, 0.3, size=(H, W))
    delta = np.array([0.0, 0.05, 0.13, 0.26, 0.31, 0.12, 0.02, -0.11, -0.35, -0.3, 0.0, 0.07])[:T]
    E = (np.exp(y0[None] + delta[:, None, None]) - 1e-3).astype(np.float32)
    return E, feat, delta


def test_new_window_sees_a_global_brightness_change():
    """Features static, y_t = y_0 + delta_t, single-frame windows: the new
    window fires eq. (1) on delta_t at every pixel; the features-driven forms
    fire nothing (the limitation of a threshold that only sees features)."""
    E, feat, delta = _flicker()
    T, F, H, W = feat.shape
    C = 0.2
    say("flicker scene, explicit new window")
    expect = []
    ref = delta[0]
    for t in range(1, T):
        d = delta[t] - ref
        if abs(d) >= C:
            expect.append((t, 1 if d > 0 else -1))
            ref = delta[t]
    assert expect
    ev, _ = run_gpu(E, feat, B.Params(r=2, tr=0, C=C, threshold=B.THRESHOLD_NEW_WINDOW), "thresholded")
    assert ev["count"] == len(expect) * H * W
    got = sorted(set(zip(ev["t"].tolist(), ev["p"].tolist())))
    assert got == expect
    for t, _ in expect:
        assert np.sum(ev["t"] == t) == H * W
    for thr in (B.THRESHOLD_CLOSED, B.THRESHOLD_LAST_WINDOW):
        ev, _ = run_gpu(E, feat, B.Params(r=2, tr=0, C=C, threshold=thr), "thresholded")
        assert ev["count"] == 0, thr


@pytest.mark.parametrize("form", ["last", "new"])
def test_explicit_step_equals_separate_calls_and_graph(small_clip, form):
    """esim_step (threshold, compaction, work-list regression, state update)
    equals the separate calls bit for bit, and graph replays reproduce it."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    p = _params(cfg, form)
    say(f"explicit {form}: step vs separate calls, graph")
    y, fd = to_dev(E, feat)
    a = Simulator(y, fd, p)
    b = Simulator(y, fd, p)
    ea = a.run("thresholded", fused=True)
    eb = b.run("thresholded", fused=False)
    assert ea["count"] == eb["count"] > 0
    for k in ("x", "y", "t", "p"):
        assert np.array_equal(ea[k], eb[k]), k
    for k in ("alpha", "beta", "xref", "tref", "bxy"):
        assert torch.equal(getattr(a.state, k), getattr(b.state, k)), k
    assert torch.equal(a.state.rmom, b.state.rmom)
    a.capture("thresholded")
    for _ in range(2):
        a.replay()
        torch.cuda.synchronize()
        g = a.events()
        for k in ("x", "y", "t", "p"):
            assert np.array_equal(g[k], ea[k]), k
        _ = (y * 2).sum().item()


@pytest.mark.parametrize("missing", ["bxy", "rmom"])
def test_explicit_needs_the_whole_plane(small_clip, missing):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    say(f"explicit threshold without {missing}")
    y, fd = to_dev(E, feat)
    T, F, H, W = feat.shape
    st = B.State(H, W, F, fd.device)
    setattr(st, missing, None)
    plan = B.Plan([y], [fd], [_params(cfg, "new")], [st])
    dl = torch.empty(H * W, device=fd.device)
    wl = torch.empty(H * W, dtype=torch.int64, device=fd.device)
    cnt = torch.zeros(2, dtype=torch.int32, device=fd.device)
    a = torch.empty(H * W, device=fd.device)
    b = torch.empty((F + 2, H * W), device=fd.device)
    with pytest.raises(B.EsimError):
        B.threshold(plan, 1, dl, wl, cnt)
    with pytest.raises(B.EsimError):
        B.step(plan, 0, B.INIT)
    with pytest.raises(B.EsimError):
        B.events(plan, 0, B.INIT, None, alpha=a, beta=b, n_out=H * W)


@pytest.mark.parametrize("form", ["last", "new"])
def test_explicit_batch_equals_single_clips(form):
    """A plan of clips of uneven size, length and radius: a work list (and the
    window sums over it) then spans several clips; every clip's events equal
    its own single-clip run, fused and unfused."""
    from paper_2303_02608_amd.simulator import BatchSimulator
    say(f"explicit {form}: batch of uneven clips")
    shapes = [(40, 30, 9, 3, 1), (23, 57, 12, 4, 0), (64, 48, 6, 9, 1), (50, 50, 5, 2, 1)]
    clips = []
    for i, (W, H, T, r, tr) in enumerate(shapes):
        spec = synth.ClipSpec(W=W, H=H, T=T, spp=2 + i, F=7, n_discs=2 + i, speed=(0.5, 2.0),
                              seed=6000 + i)
        d = synth.make_clip(spec)
        y, fd = to_dev(d["E"].numpy(), d["feat"].numpy())
        clips.append((y, fd, B.Params(r=r, tr=tr, C=0.2, threshold=FORMS[form][0])))
    bs = BatchSimulator([c[0] for c in clips], [c[1] for c in clips], [c[2] for c in clips])
    got = bs.run()
    sep = bs.run(fused=False)
    assert got["count"] > 0
    for k in ("x", "y", "t", "p", "clip"):
        assert np.array_equal(got[k], sep[k]), k
    for c, (y, fd, p) in enumerate(clips):
        m = got["clip"] == c
        single = Simulator(y, fd, p).run("thresholded")
        for k in ("x", "y", "t", "p"):
            assert np.array_equal(got[k][m], single[k]), (c, k)


@pytest.mark.parametrize("form", ["last", "new"])
@pytest.mark.parametrize("F,feat_dtype,r,tr", [(1, "f32", 4, 1), (12, "f32", 3, 1), (7, "f16", 5, 1),
                                              (10, "f16", 8, 2)])
def test_explicit_feature_counts_and_f16(form, F, feat_dtype, r, tr):
    """The explicit forms at the extreme feature counts and with FP16 feature
    storage (the oracle decodes the same FP16 bits); r = 8 takes the work-list
    window sums over two column passes of the 16 lanes."""
    W, H, T = 48, 40, 8
    d = synth.random_features_clip(W, H, T, F, seed=70 + F, feat_dtype=feat_dtype)
    E, feat = d["E"].numpy(), d["feat"].numpy()
    p = B.Params(r=r, tr=tr, C=0.1, threshold=FORMS[form][0])
    say(f"explicit {form} F={F} {feat_dtype} r={r} tr={tr}")
    gpu, _ = run_gpu(E, feat, p, "thresholded", keep_dl=True)
    orc = oracle.run(oracle_clip(E, feat), oracle.Params(p.r, p.tr, p.C, p.h, p.b, p.ridge),
                     FORMS[form][1], want_dl=True)
    n, excused, fails = compare_events(gpu, orc, W, p.C, BAND)
    say(f"gpu {gpu['count']} oracle {orc['count']} excused {excused}")
    assert gpu["count"] > 0
    assert not fails and excused <= max(2, n // 1000), fails[:5]


@pytest.mark.parametrize("form", ["last", "new"])
def test_explicit_with_compensated_fp32_regression(small_clip, form):
    """The explicit forms over the compensated-FP32 regression (models through
    the plan's buffers at 16 and 4 lanes): the step equals the separate calls
    bit for bit and the window sums are finite."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], precision=B.GRAM_F32C, threshold=FORMS[form][0])
    say(f"explicit {form} with the compensated-FP32 regression")
    y, fd = to_dev(E, feat)
    a = Simulator(y, fd, p)
    b = Simulator(y, fd, p)
    ea = a.run("thresholded", fused=True)
    eb = b.run("thresholded", fused=False)
    assert ea["count"] == eb["count"] > 0
    for k in ("x", "y", "t", "p"):
        assert np.array_equal(ea[k], eb[k]), k
    assert torch.equal(a.state.rmom, b.state.rmom)
    assert torch.isfinite(a.state.rmom).all()


def test_explicit_batch_graph_replay():
    """A batched plan with the current-window form captured in a graph: every
    replay reproduces the eager run."""
    from paper_2303_02608_amd.simulator import BatchSimulator
    say("explicit new-window batch graph replay")
    clips = []
    for i, (W, H, T, r) in enumerate([(40, 30, 7, 3), (33, 41, 5, 4), (48, 24, 6, 2)]):
        spec = synth.ClipSpec(W=W, H=H, T=T, spp=3, F=7, n_discs=3, speed=(0.5, 2.0), seed=6100 + i)
        d = synth.make_clip(spec)
        y, fd = to_dev(d["E"].numpy(), d["feat"].numpy())
        clips.append((y, fd, B.Params(r=r, tr=1, C=0.2, threshold=B.THRESHOLD_NEW_WINDOW)))
    bs = BatchSimulator([c[0] for c in clips], [c[1] for c in clips], [c[2] for c in clips])
    eager = bs.run()
    assert eager["count"] > 0
    bs.capture()
    for _ in range(3):
        bs.graph.replay()
        torch.cuda.synchronize()
        got = bs.ev.host()
        for k in ("x", "y", "t", "p", "clip"):
            assert np.array_equal(got[k], eager[k]), k
        _ = (clips[0][0] * 2).sum().item()
