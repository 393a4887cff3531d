#!/usr/bin/env python3
"""Benchmark of the event simulator on one MI355X.

Workload: the DVS-scale clip -- 640x480 px, 120 frames at 1 ms, 8 spp
exponential-noise radiance, 7 FP32 feature channels (normal, albedo, depth),
window radius 7, temporal radius 1, C = 0.15 -- drawn by the seeded
procedural generator directly in HBM.

A step is one whole conversion of the clip: log brightness, then the paper's
thresholded path (regress all pixels at frame 0; per frame threshold,
compaction, regression of the flagged pixels, events).  The step is captured
once in a hipGraph and replayed.  The exhaustive WLR+ESIM path is timed the
same way on the same clip.  `value` is the thresholded path's pixel-frames/s
(T*H*W per step); events/s are reported beside it.

Other workloads (`--workload`, one JSON line each; the default is the DVS line
above): `precision` (1920x1080, F = 10 FP16 features, r = 10, tr = 2: dense
regression and a 24-frame thresholded conversion with the FP64 Gram and with
the compensated-FP32 Gram), `batch` (the 32-clip batch, frames scaled down to
about 2e8 pixel-frames: one batched plan against the clips converted one by
one) and `diff` (640x480x60: forward regressions of the differentiation loss
and their adjoint), `quality` (events of the three conversions against ESIM on
the noise-free frames: precision, recall, F1 and Chamfer distance over a sweep
of C, with the conversion times), `threshold` (the closed form of Prop. 1
against the explicit Delta R sums over the last-event window and over the
current frame's window: times, events and quality, on the clip and under a
global illumination flicker), `bandwidth` (WLR+ESIM and the thresholded method
with the regression bandwidth chosen per regression by SURE from the MC
variance, against the plain regressions), `multicrossing` (raw and WLR+ESIM
with every crossing against one event per pixel-frame, scored against
every-crossing ESIM on the noise-free frames, with the comparison's own time).

Roofline: the dominant kernel is the regression.  Its launches are bracketed
with HIP events on the launch stream during an instrumented eager pass of the
same conversion; achieved = algorithmic FLOPs (per regression
|Omega| (P^2 + 4P + 4D) + P^3/3 + 2P^2, with the truncated window size) / the
summed launch durations.  The CPU baseline is the FP64 oracle on a random
sample of pixels of the same clip (all frames), on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel-frames/s and events/s, thresholded vs exhaustive WLR, same MI355X"
PEAK_ALU_TFLOPS = 78.6      # FP64 vector (= unpacked FP32) issue peak of MI355X
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def omega_sizes(x, y, t, W, H, T, r, tr):
    """Truncated window size |Omega| of regressions centred at (x, y, t)."""
    nx = np.minimum(x + r, W - 1) - np.maximum(x - r, 0) + 1
    ny = np.minimum(y + r, H - 1) - np.maximum(y - r, 0) + 1
    nt = np.minimum(t + tr, T - 1) - np.maximum(t - tr, 0) + 1
    return nx.astype(np.int64) * ny * nt


def regress_flops(omega, F):
    D, P = F + 2, F + 3
    return omega.astype(np.float64) * (P * P + 4 * P + 4 * D) + P ** 3 / 3.0 + 2 * P * P


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("esim_regress_impl.h", "esim_wlr.h", "esim_internal.h"):
        with open(os.path.join(ROOT, "paper_2303_02608_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(launch_items):
    """HBM bytes per launch of the regression kernel from the committed
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "regress_dvs_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def _time_ms(fn, reps, warmup=1):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _graph(fn):
    """Captures fn() (after one eager warm-up on a side stream) and returns the replay."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g.replay


def workload_precision(args, B, synth, Simulator):
    """X1: 1920x1080, all 500 frames, F = 10 FP16 features, r = 10, tr = 2:
    the FP64 Gram (production path) and the compensated FP32 Gram with an FP64
    re-solve above the equilibrated condition bound 1e6."""
    import torch
    from paper_2303_02608_amd import autotune
    cfg = synth.config_spec(4)
    spec = cfg["spec"]
    T = spec.T if args.precision_frames is None else args.precision_frames
    t0 = time.time()
    H, W, F = spec.H, spec.W, spec.F
    y = torch.empty((T, H, W), dtype=torch.float32, device="cuda")
    feat = torch.empty((T, F, H, W), dtype=torch.float16, device="cuda")
    step = 25
    for a in range(0, T, step):
        b = min(T, a + step)
        d = synth.make_clip(spec, device="cuda", frames=range(a, b))
        B.log_brightness(d["E"], out=y[a:b])
        feat[a:b].copy_(d["feat"])
        del d
        torch.cuda.synchronize()
        log(f"generated frames {a}..{b - 1} of {T} ({time.time() - t0:.0f}s)")
    HW = H * W
    r, tr, C = cfg["r"], cfg["tr"], cfg["C"]
    tc = T // 2
    om = omega_sizes(np.arange(HW) % W, np.arange(HW) // W, np.full(HW, tc), W, H, T, r, tr)
    fl = regress_flops(om, F).sum()
    out = {"workload": f"precision {W}x{H}x{T}, F={F} f16, r={r}, tr={tr}, C={C}",
           "generate_s": round(time.time() - t0, 1)}
    for name, prec, kb in (("fp64", B.GRAM_F64, float("inf")), ("f32c", B.GRAM_F32C, 1e6)):
        p = B.Params(r=r, tr=tr, C=C, precision=prec, kappa_fp64=kb, dt=cfg["dt"])
        sim = Simulator(y, feat, p)
        plan = sim.plan
        sched = autotune.tune(plan)
        a = torch.empty(HW, device="cuda")
        bb = torch.empty((plan.D, HW), device="cuda")
        ms = _time_ms(lambda: B.regress(plan, tc, None, None, HW, a, bb), 3)
        row = {"dense_regress_ms": round(ms, 3), "dense_tflops": round(fl / (ms * 1e-3) / 1e12, 2),
               "dense_frac": round(fl / (ms * 1e-3) / 1e12 / PEAK_ALU_TFLOPS, 4),
               "schedule": list(sched)}
        if prec == B.GRAM_F32C:
            # share of regressions re-solved in FP64 (equilibrated kappa-hat
            # above the bound), every pixel of the first, middle and last frames
            K = torch.empty(HW, device="cuda")
            shares = {}
            for t in (tr, tc, T - 1 - tr):
                B.regress(plan, t, None, None, HW, a, bb, None, K)
                k = K.cpu().numpy()
                shares[str(t)] = round(float(np.mean(~(k <= kb))), 6)
                if t == tc:
                    row["kappa_hat_quantiles"] = {q: float(np.quantile(k[np.isfinite(k)], q))
                                                  for q in (0.5, 0.9, 0.99, 0.999)}
            row["fp64_resolve_share"] = shares
        run = _graph(lambda: sim.enqueue("thresholded"))
        ms_t = _time_ms(run, 2)
        ev = sim.events()
        row.update(thresholded_ms=round(ms_t, 3), pixel_frames_per_s=round(T * HW / (ms_t * 1e-3), 1),
                   events=ev["count"], events_per_s=round(ev["count"] / (ms_t * 1e-3), 1),
                   flagged_fraction=round(ev["count"] / ((T - 1) * HW), 5))
        out[name] = row
        log(f"precision {name}: dense {ms:.3f} ms, thresholded {ms_t:.3f} ms")
        del sim, plan
        torch.cuda.empty_cache()
    return out


def workload_batch(args, B, synth, Simulator):
    """X2: the 32-clip batch at its full size (every clip's T frames), one plan
    and one persistent work-list launch per step over all clips, against the
    same clips converted one plan each; per-clip flagged fraction reported."""
    import torch
    from paper_2303_02608_amd.simulator import BatchSimulator
    specs = synth.batch_specs(32, seed=5000)
    t0 = time.time()
    ys, feats, params = [], [], []
    for k, c in enumerate(specs):
        d = synth.make_clip(c["spec"], device="cuda")
        ys.append(B.log_brightness(d["E"]))
        feats.append(d["feat"])
        params.append(B.Params(r=c["r"], tr=c["tr"], C=c["C"], dt=c["dt"]))
        del d
        torch.cuda.synchronize()
        log(f"generated clip {k}: {c['spec'].W}x{c['spec'].H}x{c['spec'].T} ({time.time() - t0:.0f}s)")
    pf = sum(int(f.shape[0]) * f.shape[2] * f.shape[3] for f in feats)
    log(f"generated {len(specs)} clips, {pf / 1e6:.1f} M pixel-frames in {time.time() - t0:.1f}s")
    bs = BatchSimulator(ys, feats, params)
    run = _graph(bs.enqueue)
    ms_b = _time_ms(run, 3)
    got = bs.ev.host()
    ev_b = got["count"]
    log(f"batch: {ms_b:.2f} ms batched")
    clips = []
    for k, (c, f) in enumerate(zip(specs, feats)):
        T, F, H, W = f.shape
        n = int((got["clip"] == k).sum())
        clips.append({"W": W, "H": H, "T": T, "spp": c["spec"].spp, "r": c["r"],
                      "phi_target": round(c["phi_target"], 4),
                      "phi": round(n / max(1, (T - 1) * H * W), 4), "events": n})
    del bs
    sims = [Simulator(y, f, p) for y, f, p in zip(ys, feats, params)]
    runs = [_graph(lambda s=s: s.enqueue("thresholded")) for s in sims]
    ms_s = _time_ms(lambda: [r() for r in runs], 3)
    ev_s = sum(s.events()["count"] for s in sims)
    log(f"batch: {ms_b:.2f} ms batched, {ms_s:.2f} ms one by one")
    phis = [c["phi"] for c in clips]
    return {"workload": f"batch of {len(specs)} clips, {pf} pixel-frames (every clip at its full length)",
            "pixel_frames": pf,
            "batched_ms": round(ms_b, 3), "batched_pixel_frames_per_s": round(pf / (ms_b * 1e-3), 1),
            "one_by_one_ms": round(ms_s, 3),
            "one_by_one_pixel_frames_per_s": round(pf / (ms_s * 1e-3), 1),
            "events": ev_b, "events_one_by_one": ev_s,
            "batched_speedup": round(ms_s / ms_b, 3),
            "phi_range": [min(phis), max(phis)], "clips": clips}


def workload_diff(args, B, synth, Simulator):
    """X3: forward regressions of the differentiation loss and their adjoint."""
    import torch
    cfg = synth.config_spec(3)
    spec = cfg["spec"]
    t0 = time.time()
    d = synth.make_clip(spec, device="cuda")
    y = B.log_brightness(d["E"])
    feat = d["feat"]
    torch.cuda.synchronize()
    log(f"generated {spec.W}x{spec.H}x{spec.T} in {time.time() - t0:.1f}s")
    T, F, H, W = feat.shape
    HW = H * W
    r, tr, C = cfg["r"], cfg["tr"], cfg["C"]
    p = B.Params(r=r, tr=tr, C=C)
    ev = Simulator(y, feat, p).run("thresholded")
    xs, ys_, ts = (ev[k].astype(np.int64) for k in ("x", "y", "t"))
    items = np.concatenate([np.arange(HW, dtype=np.int64), (ts << 44) | (ys_ * W + xs)])
    n = items.size
    it = torch.from_numpy(items).cuda()
    plan = B.Plan([y], [feat], [p])
    alpha = torch.empty(n, device="cuda")
    cnt = torch.tensor([n, n], dtype=torch.int32, device="cuda")
    ms_f = _time_ms(lambda: B.regress(plan, -1, it, cnt, n, alpha), 3)
    g_a = torch.ones(n, device="cuda")
    g_y = torch.zeros_like(y)
    g_b = torch.zeros(plan.D, dtype=torch.float64, device="cuda")
    scratch = torch.empty(B.backward_scratch_bytes(plan, n), dtype=torch.uint8, device="cuda")
    ms_b = _time_ms(lambda: B.backward(plan, it, g_a, g_y, g_b, scratch), 3)
    tt = np.concatenate([np.zeros(HW, np.int64), ts])
    px = np.concatenate([np.arange(HW) % W, xs])
    py = np.concatenate([np.arange(HW) // W, ys_])
    om = omega_sizes(px, py, tt, W, H, T, r, tr)
    fl_f = regress_flops(om, F).sum()
    fl_b = fl_f + 60.0 * om.sum()     # the adjoint recomputes the forward window, then ~60 FLOP/sample
    log(f"diff: {n} regressions, forward {ms_f:.2f} ms, adjoint {ms_b:.2f} ms")
    return {"workload": f"diff {W}x{H}x{T}, F={F}, r={r}, tr={tr}, C={C}",
            "regressions": int(n), "forward_ms": round(ms_f, 3),
            "forward_regressions_per_s": round(n / (ms_f * 1e-3), 1),
            "forward_tflops": round(fl_f / (ms_f * 1e-3) / 1e12, 2),
            "adjoint_ms": round(ms_b, 3), "adjoint_regressions_per_s": round(n / (ms_b * 1e-3), 1),
            "adjoint_tflops": round(fl_b / (ms_b * 1e-3) / 1e12, 2),
            "adjoint_flop_model": "forward F_reg + 60 FLOP per window sample"}


EDGE_PX = 1.5    # an event within this distance of a disc outline is at a moving edge


PLACES = ("edge", "near", "interior")


def place_classes(spec, t, x, y, r):
    """Place of events at (t, x, y): 0 "edge" (the pixel centre within EDGE_PX
    of a disc outline at frame t or t - 1, so a moving outline crossed or
    touched the pixel), 1 "near" (within r: the regression window reaches an
    outline), 2 "interior"."""
    import torch
    from paper_2303_02608_amd import synth
    t, x, y = t.long(), x.long(), y.long()
    dist = torch.minimum(synth.boundary_distance(spec, t, x, y),
                         synth.boundary_distance(spec, (t - 1).clamp(min=0), x, y))
    return torch.where(dist <= EDGE_PX, 0, torch.where(dist <= r, 1, 2))


def edge_split(spec, ev, d, r, taus):
    """Events split by place (place_classes).  Per class: the events and the
    share whose nearest same-polarity counterpart is closer than each tau
    (precision for generated events, recall for reference events)."""
    cls = place_classes(spec, ev["t"], ev["x"], ev["y"], r)
    out = {}
    for k, name in enumerate(PLACES):
        m = cls == k
        n = int(m.sum())
        out[name] = {"events": n,
                     "share": [round(float((d[m] < tau).double().mean()), 4) if n else None
                               for tau in taus]}
    return out


def prediction_check(sim, spec, r, C):
    """The thresholded path's predicted change against the change its new
    regression shows, per event.  A pixel fires when the predicted change
    dL = beta_ref^T (f_t - x_ref) reaches C; the regression at the event then
    gives alpha_t, and alpha_t - alpha_ref is the change of the fitted value.
    Per place: the events, the median of (alpha_t - alpha_ref) / dL, the share
    whose fitted change is below C / 2 in the predicted direction, and the
    share whose fitted change has the opposite sign."""
    import torch
    from paper_2303_02608_amd import binding as B
    p, n, T, W = sim.plan, sim.HW, sim.T, sim.W
    B.regress(p, 0, None, None, n, sim.alpha, sim.beta)
    B.events(p, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=n)
    sim.ev.count.zero_()
    ts, xs, ys, pred, act = [], [], [], [], []
    for t in range(1, T):
        B.threshold(p, t, sim.dl, sim.worklist, sim.count)
        B.regress(p, t, sim.worklist, sim.count, n, sim.alpha, sim.beta)
        m = int(sim.count[0].item())
        pix = sim.worklist[:m] & 0xFFFFFFFF
        pred.append(sim.dl[pix].double())
        act.append(sim.alpha[:m].double() - sim.state.alpha[pix].double())
        ts.append(torch.full_like(pix, t))
        xs.append(pix % W)
        ys.append(pix // W)
        B.events(p, t, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count,
                 dl=sim.dl, alpha=sim.alpha, beta=sim.beta, n_out=n)
    t, x, y = torch.cat(ts), torch.cat(xs), torch.cat(ys)
    pred, act = torch.cat(pred), torch.cat(act)
    along = act * torch.sign(pred)                 # fitted change in the predicted direction
    cls = place_classes(spec, t, x, y, r)
    out = {}
    for k, name in enumerate(PLACES):
        mk = cls == k
        nk = int(mk.sum())
        if nk == 0:
            out[name] = {"events": 0}
            continue
        out[name] = {"events": nk,
                     "median_fitted_over_predicted": round(float((act[mk] / pred[mk]).median()), 4),
                     "below_half_C": round(float((along[mk] < 0.5 * C).double().mean()), 4),
                     "opposite_sign": round(float((along[mk] < 0).double().mean()), 4)}
    return out


def workload_quality(args, B, synth, Simulator):
    """Event quality against ESIM on the noise-free frames of the DVS clip
    (Sec. 3 "Quantitative comparison", Tables 1 and A2 on synthetic scenes),
    with conversion times, over a sweep of C."""
    import torch
    from paper_2303_02608_amd import quality as Q
    cfg = synth.config_spec(1)
    spec = cfg["spec"]
    t0 = time.time()
    d = synth.make_clip(spec, device="cuda", reference=True)
    y = B.log_brightness(d["E"])
    y_ref = B.log_brightness(d["E_ref"])
    feat = d["feat"]
    torch.cuda.synchronize()
    log(f"generated {spec.W}x{spec.H}x{spec.T} with reference frames in {time.time() - t0:.1f}s")
    T, F, H, W = feat.shape
    taus, rmax = [5e-4, 2e-3, 5e-3, 1e-2], 0.05
    rows = []
    for C in (0.15, 0.25, 0.5, 0.75, 1.0):
        p = B.Params(r=cfg["r"], tr=cfg["tr"], C=C)
        ref = Simulator(y_ref, feat, p).run("raw")
        refd = Q.to_device(ref)
        row = {"C": C, "reference_events": ref["count"]}
        for mode in ("raw", "exhaustive", "thresholded"):
            sim = Simulator(y, feat, p)
            run = _graph(lambda s=sim, m=mode: s.enqueue(m))
            ms = _time_ms(run, 2)
            ev = sim.events()
            evd = Q.to_device(ev)
            m = Q.metrics(evd, refd, W, H, T, taus, rmax, keep=True)
            row[mode] = {"ms": round(ms, 3), "events": ev["count"],
                         "P": [round(v, 4) for v in m["P"]], "R": [round(v, 4) for v in m["R"]],
                         "F": [round(v, 4) for v in m["F"]], "CD": m["CD"],
                         "precision_by_place": edge_split(spec, evd, m["dg"], cfg["r"], taus),
                         "recall_by_place": edge_split(spec, refd, m["dr"], cfg["r"], taus)}
            if mode == "thresholded":
                row[mode]["prediction_by_place"] = prediction_check(sim, spec, cfg["r"], C)
            del sim, run
            log(f"C={C} {mode}: {ms:.2f} ms, {ev['count']} events, F {row[mode]['F']}")
        rows.append(row)
    return {"workload": f"quality DVS {W}x{H}x{T}, r={cfg['r']}, tr={cfg['tr']}; reference = ESIM on the "
                        f"noise-free frames; coordinates normalised by (W, H, T)",
            "taus": taus, "rmax": rmax, "sweep": rows}


def window_sum_flops(om, F):
    """Algorithmic FLOPs of one window pass of the explicit thresholds (W,
    sum w r, sum w r^2 of a stored plane), per window sample: the eq. (5)
    exponent over the D regressors (2F scaled feature offsets, 2D squares),
    the plane's residual (2D + 1) and the sums (5)."""
    D = F + 2
    return om.astype(np.float64) * (2 * F + 4 * D + 6)


def workload_threshold(args, B, synth, Simulator):
    """The three threshold forms of Sec. 2.2 on the DVS clip: the closed form
    of Prop. 1 and the explicit sums of eq. (7) over the last-event window and
    over the current frame's window.  Per form: conversion time, flagged
    pixels, events and their quality against ESIM on the noise-free frames, on
    the clip as generated and with a global illumination flicker (a gain on
    every pixel, the features unchanged) applied to both; plus the explicit
    threshold launches timed with HIP events on their stream."""
    import torch
    from paper_2303_02608_amd import quality as Q
    cfg = synth.config_spec(1)
    spec = cfg["spec"]
    t0 = time.time()
    d = synth.make_clip(spec, device="cuda", reference=True)
    feat = d["feat"]
    T, F, H, W = feat.shape
    HW = H * W
    r, tr, C = cfg["r"], cfg["tr"], cfg["C"]
    log(f"generated {W}x{H}x{T} with reference frames in {time.time() - t0:.1f}s")
    taus, rmax = [5e-4, 2e-3, 5e-3, 1e-2], 0.05
    tt = torch.arange(T, device="cuda", dtype=torch.float32)
    gain = torch.exp(0.3 * torch.sin(2 * np.pi * tt / 40.0))[:, None, None]
    scenes = {"as_generated": (d["E"], d["E_ref"]), "flicker": (d["E"] * gain, d["E_ref"] * gain)}
    xs, ys = np.arange(HW) % W, np.arange(HW) // W
    forms = (("closed", B.THRESHOLD_CLOSED), ("last_window", B.THRESHOLD_LAST_WINDOW),
             ("new_window", B.THRESHOLD_NEW_WINDOW))
    out = {"workload": f"threshold forms, DVS {W}x{H}x{T}, F={F} f32, r={r}, tr={tr}, C={C}; "
                       f"reference = ESIM on the noise-free frames; flicker = gain "
                       f"exp(0.3 sin(2 pi t / 40)) on every pixel",
           "taus": taus, "rmax": rmax}
    stream = torch.cuda.current_stream()
    for sname, (E, Eref) in scenes.items():
        y = B.log_brightness(E.contiguous())
        yref = B.log_brightness(Eref.contiguous())
        p0 = B.Params(r=r, tr=tr, C=C)
        refd = Q.to_device(Simulator(yref, feat, p0).run("raw"))
        rows = {}
        for name, thr in forms:
            p = B.Params(r=r, tr=tr, C=C, threshold=thr)
            sim = Simulator(y, feat, p)
            run = _graph(lambda s=sim: s.enqueue("thresholded"))
            ms = _time_ms(run, max(1, args.steps))
            ev = sim.events()
            m = Q.metrics(Q.to_device(ev), refd, W, H, T, taus, rmax)
            row = {"ms": round(ms, 3), "pixel_frames_per_s": round(T * HW / (ms * 1e-3), 1),
                   "events": ev["count"], "flagged_fraction": round(ev["count"] / ((T - 1) * HW), 5),
                   "P": [round(v, 4) for v in m["P"]], "R": [round(v, 4) for v in m["R"]],
                   "F": [round(v, 4) for v in m["F"]], "CD": m["CD"]}
            if thr != B.THRESHOLD_CLOSED and sname == "as_generated":
                # separate calls: the threshold launch (explicit kernel + compaction) and the
                # event call (events, state update and the window sums of the new planes)
                plan = sim.plan
                sim.ev.count.zero_()
                B.regress(plan, 0, None, None, HW, sim.alpha, sim.beta)
                B.events(plan, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=HW)
                th_marks, ev_marks = [], []
                for t in range(1, T):
                    marks = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                    marks[0].record(stream)
                    B.threshold(plan, t, sim.dl, sim.worklist, sim.count)
                    marks[1].record(stream)
                    B.regress(plan, t, sim.worklist, sim.count, HW, sim.alpha, sim.beta)
                    marks[2].record(stream)
                    B.events(plan, t, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count,
                             dl=sim.dl, alpha=sim.alpha, beta=sim.beta, n_out=HW)
                    marks[3].record(stream)
                    th_marks.append((marks[0], marks[1]))
                    ev_marks.append((marks[2], marks[3]))
                torch.cuda.synchronize()
                th_ms = np.array([a.elapsed_time(b) for a, b in th_marks])
                ev_ms = np.array([a.elapsed_time(b) for a, b in ev_marks])
                upd = sim.events()
                om_upd = omega_sizes(upd["x"].astype(np.int64), upd["y"].astype(np.int64),
                                     upd["t"].astype(np.int64), W, H, T, r, tr)
                fl_upd = window_sum_flops(om_upd, F).sum()
                if thr == B.THRESHOLD_LAST_WINDOW:
                    # state beta, xref, rmom and the frame's features read, dl written
                    nbytes = HW * ((3 * F + 2) * 4 + 4)
                    ach = nbytes / (th_ms.mean() * 1e-3) / 1e9
                    roofl = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                             "bytes_per_launch": nbytes}
                else:
                    fl = sum(window_sum_flops(omega_sizes(xs, ys, np.full(HW, t), W, H, T, r, tr),
                                              F).sum() for t in range(1, T))
                    ach = fl / (th_ms.sum() * 1e-3) / 1e12
                    roofl = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_ALU_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(ach / PEAK_ALU_TFLOPS, 4),
                             "flop_per_launch": float(fl / th_ms.size)}
                form = "new" if thr == B.THRESHOLD_NEW_WINDOW else "last"
                row["threshold_launch"] = {
                    "kernel": f"explicit_flag_kernel<F={F},f32,{form}> + compaction",
                    "launches": int(th_ms.size), "avg_ms": round(float(th_ms.mean()), 4),
                    "roofline": roofl, "share_of_conversion": round(float(th_ms.sum()) / ms, 3)}
                row["update_launch"] = {
                    "kernels": "events + state update + moments_kernel (16 lanes per item)",
                    "launches": int(ev_ms.size), "avg_ms": round(float(ev_ms.mean()), 4),
                    "window_sum_tflops": round(fl_upd / (ev_ms.sum() * 1e-3) / 1e12, 3),
                    "share_of_conversion": round(float(ev_ms.sum()) / ms, 3)}
                log(f"{name}: threshold launches avg {th_ms.mean():.4f} ms ({roofl['frac']:.3f} of peak), "
                    f"event calls avg {ev_ms.mean():.4f} ms")
            rows[name] = row
            log(f"{sname} {name}: {ms:.2f} ms, {ev['count']} events, F {row['F']}")
            del sim, run
        out[sname] = rows
    return out


def workload_bandwidth(args, B, synth, Simulator):
    """Bandwidth optimisation (Sec. 3): the DVS clip converted by WLR+ESIM and by
    the thresholded method with the regression's global bandwidth h chosen per
    regression among HS by SURE with the MC variance, against the plain
    regressions (h = 1): times, the chosen-h shares, and event quality against
    ESIM on the noise-free frames."""
    import torch
    from paper_2303_02608_amd import quality as Q
    cfg = synth.config_spec(1)
    spec = cfg["spec"]
    HS = [0.5, 0.75, 1.0, 1.5, 2.0]
    t0 = time.time()
    d = synth.make_clip(spec, device="cuda", reference=True)
    feat = d["feat"]
    T, F, H, W = feat.shape
    HW = H * W
    r, tr, C = cfg["r"], cfg["tr"], cfg["C"]
    y = B.log_brightness(d["E"])
    vy = B.log_variance(d["E"], d["var"], spec.spp)
    yref = B.log_brightness(d["E_ref"])
    log(f"generated {W}x{H}x{T} with variance and reference frames in {time.time() - t0:.1f}s")
    p = B.Params(r=r, tr=tr, C=C)
    refd = Q.to_device(Simulator(yref, feat, p).run("raw"))
    taus, rmax = [5e-4, 2e-3, 5e-3, 1e-2], 0.05
    sim = Simulator(y, feat, p)
    plan, n = sim.plan, HW
    hsel = torch.empty(HW, device="cuda")
    counts = torch.zeros((T, len(HS)), dtype=torch.int64, device="cuda")
    hs_t = torch.tensor(HS, device="cuda")

    def exhaustive_bw():
        sim.ev.count.zero_()
        for t in range(T):
            B.regress_bandwidth(plan, t, None, None, n, vy, HS, sim.alpha, None, hsel)
            B.events(plan, t, B.EXHAUSTIVE, sim.ev, dl=sim.dl, alpha=sim.alpha, n_out=n)

    def thresholded_bw():
        sim.ev.count.zero_()
        B.regress_bandwidth(plan, 0, None, None, n, vy, HS, sim.alpha, sim.beta, hsel)
        B.events(plan, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=n)
        for t in range(1, T):
            B.threshold(plan, t, sim.dl, sim.worklist, sim.count)
            B.regress_bandwidth(plan, t, sim.worklist, sim.count, n, vy, HS, sim.alpha, sim.beta)
            B.events(plan, t, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count, dl=sim.dl,
                     alpha=sim.alpha, beta=sim.beta, n_out=n)

    out = {"workload": f"bandwidth optimisation, DVS {W}x{H}x{T}, F={F} f32, r={r}, tr={tr}, C={C}; "
                       f"candidates h = {HS} chosen by SURE with the MC variance; reference = ESIM on "
                       f"the noise-free frames", "taus": taus, "rmax": rmax}
    runs = {"exhaustive_plain": lambda: sim.enqueue("exhaustive"),
            "exhaustive_bandwidth": exhaustive_bw,
            "thresholded_plain": lambda: sim.enqueue("thresholded"),
            "thresholded_bandwidth": thresholded_bw}
    for name, fn in runs.items():
        run = _graph(fn)
        ms = _time_ms(run, max(1, args.steps))
        ev = sim.events()
        m = Q.metrics(Q.to_device(ev), refd, W, H, T, taus, rmax)
        out[name] = {"ms": round(ms, 3), "pixel_frames_per_s": round(T * HW / (ms * 1e-3), 1),
                     "events": ev["count"], "P": [round(v, 4) for v in m["P"]],
                     "R": [round(v, 4) for v in m["R"]], "F": [round(v, 4) for v in m["F"]], "CD": m["CD"]}
        log(f"{name}: {ms:.2f} ms, {ev['count']} events, F {out[name]['F']}")
        del run
    # the dense bandwidth launch alone, with the chosen-h shares over the clip
    stream = torch.cuda.current_stream()
    marks = []
    for t in range(T):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.regress_bandwidth(plan, t, None, None, n, vy, HS, sim.alpha, None, hsel)
        e1.record(stream)
        marks.append((e0, e1))
        counts[t] = (hsel[:, None] == hs_t[None, :]).sum(dim=0)
    torch.cuda.synchronize()
    dms = np.array([a.elapsed_time(b) for a, b in marks])
    fl = 0.0
    xs, ys = np.arange(HW) % W, np.arange(HW) // W
    for t in range(T):
        fl += len(HS) * regress_flops(omega_sizes(xs, ys, np.full(HW, t), W, H, T, r, tr), F).sum()
    ach = fl / (dms.sum() * 1e-3) / 1e12
    share = (counts.sum(dim=0).double() / (T * HW)).cpu().numpy()
    out["dense_launch"] = {"kernel": f"bandwidth_kernel<F={F},f32>", "candidates": len(HS),
                           "avg_ms": round(float(dms.mean()), 4),
                           "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_ALU_TFLOPS,
                                        "unit": "TFLOP/s", "frac": round(ach / PEAK_ALU_TFLOPS, 4),
                                        "flop_model": "candidates x F_reg per regression"},
                           "chosen_h_share": {str(h): round(float(v), 4) for h, v in zip(HS, share)}}
    log(f"dense bandwidth launch avg {dms.mean():.3f} ms ({ach:.1f} TFLOP/s); h shares {share}")
    return out


def workload_multicrossing(args, B, synth, Simulator):
    """Every-crossing ESIM (the multi_crossing option) on the DVS clip: raw and
    WLR+ESIM conversions with one event per pixel-frame and with every
    crossing, their times, and their quality against every-crossing ESIM on the
    noise-free frames; plus the event-set comparison's own time (the GPU
    nearest-neighbour search of both directions)."""
    import torch
    from paper_2303_02608_amd import quality as Q
    cfg = synth.config_spec(1)
    spec = cfg["spec"]
    t0 = time.time()
    d = synth.make_clip(spec, device="cuda", reference=True)
    feat = d["feat"]
    T, F, H, W = feat.shape
    r, tr, C = cfg["r"], cfg["tr"], cfg["C"]
    y = B.log_brightness(d["E"])
    yref = B.log_brightness(d["E_ref"])
    log(f"generated {W}x{H}x{T} with reference frames in {time.time() - t0:.1f}s")
    taus, rmax = [5e-4, 2e-3, 5e-3, 1e-2], 0.05
    pm = B.Params(r=r, tr=tr, C=C, multi_crossing=True)
    ref = Simulator(yref, feat, pm, capacity=1 << 27).run("raw")
    refd = Q.to_device(ref)
    out = {"workload": f"every-crossing ESIM, DVS {W}x{H}x{T}, r={r}, tr={tr}, C={C}; reference = "
                       f"every-crossing ESIM on the noise-free frames ({ref['count']} events)",
           "taus": taus, "rmax": rmax}
    stream = torch.cuda.current_stream()
    for mode in ("raw", "exhaustive"):
        for multi in (False, True):
            p = B.Params(r=r, tr=tr, C=C, multi_crossing=multi)
            sim = Simulator(y, feat, p, capacity=1 << 27)
            run = _graph(lambda s=sim, m=mode: s.enqueue(m))
            ms = _time_ms(run, max(1, args.steps))
            ev = sim.events()
            evd = Q.to_device(ev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            m = Q.metrics(evd, refd, W, H, T, taus, rmax)
            e1.record(stream)
            torch.cuda.synchronize()
            key = f"{mode}_{'every_crossing' if multi else 'one_per_frame'}"
            out[key] = {"ms": round(ms, 3), "pixel_frames_per_s": round(T * H * W / (ms * 1e-3), 1),
                        "events": ev["count"], "F": [round(v, 4) for v in m["F"]], "CD": m["CD"],
                        "metrics_ms": round(e0.elapsed_time(e1), 3)}
            log(f"{key}: {ms:.2f} ms, {ev['count']} events, F {out[key]['F']}, "
                f"metrics {out[key]['metrics_ms']} ms")
            del sim, run
    return out


KAPPA_DECADES = 13   # kappa-hat histogram bins: [10^k, 10^(k+1)) for k < 12, then >= 1e12


def kappa_histogram(k):
    """Counts of kappa-hat per decade (KAPPA_DECADES bins from 1) and of
    non-finite values."""
    fin = np.isfinite(k)
    e = np.clip(np.floor(np.log10(np.maximum(k[fin], 1.0))), 0, KAPPA_DECADES - 1).astype(np.int64)
    return np.bincount(e, minlength=KAPPA_DECADES), int((~fin).sum())


def frame_log(sim, feat, params, emit):
    """Per-frame record of one thresholded conversion, run untimed after the
    timed steps: the flagged fraction and events of each frame, the number of
    regressions re-solved in FP64 (compensated FP32 Gram only), a histogram of
    the equilibrated condition estimate of the frame's regressions, and the
    stuck pixels -- those whose stored gradient cannot reach the threshold for
    any feature change within the clip's own feature range
    (sum_j |beta_ref_j| span_j < C, so |dL| = |beta_ref^T (f - x_ref)| < C
    forever).  emit(dict) receives one record per frame; the summary is
    returned."""
    import torch
    from paper_2303_02608_amd import binding as B
    p, n, T = sim.plan, sim.HW, sim.T
    f32 = feat.float() if feat.dtype != torch.float32 else feat
    span = torch.stack([(f32[:, j].amax() - f32[:, j].amin()) for j in range(sim.F)]).view(-1, 1)
    del f32
    kap = torch.empty(n, dtype=torch.float32, device=feat.device)
    a2 = torch.empty(n, dtype=torch.float32, device=feat.device)
    c32 = params.precision == B.GRAM_F32C
    bound = params.kappa_fp64
    hist_all = np.zeros(KAPPA_DECADES, np.int64)
    nonfin_all = resolves_all = 0
    phis, stucks = [], []

    def stuck():
        return int(((sim.state.beta.abs() * span).sum(0) < params.C).sum())

    def kappas(t, wl, cnt, m):
        B.regress(p, t, wl, cnt, n, a2, None, None, kap)
        k = kap[:m].cpu().numpy().astype(np.float64)
        h, nf = kappa_histogram(k)
        res = int(np.sum(~(k <= bound))) if c32 else 0
        return h, nf, res, float(np.max(k)) if k.size else 0.0

    sim.ev.count.zero_()
    B.regress(p, 0, None, None, n, sim.alpha, sim.beta)
    B.events(p, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=n)
    h, nf, res, kmax = kappas(0, None, None, n)
    hist_all += h
    nonfin_all += nf
    resolves_all += res
    s = stuck()
    stucks.append(s)
    emit({"frame": 0, "regressions": n, "fp64_resolves": res, "kappa_hist": h.tolist(),
          "kappa_nonfinite": nf, "kappa_max": kmax, "stuck": s})
    ev_prev = 0
    for t in range(1, T):
        B.threshold(p, t, sim.dl, sim.worklist, sim.count)
        B.regress(p, t, sim.worklist, sim.count, n, sim.alpha, sim.beta)
        m = int(sim.count[1].item())
        h, nf, res, kmax = kappas(t, sim.worklist, sim.count, m)
        B.events(p, t, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count,
                 dl=sim.dl, alpha=sim.alpha, beta=sim.beta, n_out=n)
        ev = int(sim.ev.count[0].item())
        s = stuck()
        hist_all += h
        nonfin_all += nf
        resolves_all += res
        phis.append(m / n)
        stucks.append(s)
        emit({"frame": t, "flagged": m, "phi": round(m / n, 6), "events": ev - ev_prev,
              "fp64_resolves": res, "kappa_hist": h.tolist(), "kappa_nonfinite": nf,
              "kappa_max": kmax, "stuck": s})
        ev_prev = ev
    return {"frames": T, "phi_min": round(min(phis), 6), "phi_median": round(float(np.median(phis)), 6),
            "phi_max": round(max(phis), 6), "fp64_resolves": resolves_all,
            "kappa_hist_decades_from_1": hist_all.tolist(), "kappa_nonfinite": nonfin_all,
            "stuck_first_frame": stucks[0], "stuck_last_frame": stucks[-1], "stuck_max": max(stucks),
            "precision": "compensated FP32 Gram" if c32 else "FP64 Gram (no re-solve)"}


def cpu_model():
    """The host CPU's model name (first processor of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(E, feat, r, tr, C, n_pixels):
    """The FP64 oracle, as it stands, on the host cores: the thresholded path
    over the whole clip for a random sample of pixels (their complete
    histories), scaled to pixel-frames/s.  The only use of the oracle here."""
    import oracle
    T, F, H, W = feat.shape
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rng = np.random.default_rng(1234)
    pix = np.sort(rng.choice(H * W, size=min(n_pixels, H * W), replace=False))
    oc = oracle.Clip(oracle.log_brightness(E.cpu().numpy()), feat.cpu().numpy())
    c0 = time.perf_counter()
    out = oracle.run(oc, oracle.Params(r, tr, C), oracle.THRESHOLDED, pixels=pix, nthreads=nthreads)
    secs = time.perf_counter() - c0
    log(f"oracle: {secs:.1f}s for {pix.size} px x {T} frames ({nthreads} threads)")
    # WLR+ESIM beside it: every frame of a smaller random pixel sample
    pe = np.sort(rng.choice(H * W, size=min(8000, H * W), replace=False))
    c0 = time.perf_counter()
    oe = oracle.run(oc, oracle.Params(r, tr, C), oracle.EXHAUSTIVE, pixels=pe, nthreads=nthreads)
    se = time.perf_counter() - c0
    log(f"oracle, exhaustive: {se:.1f}s for {pe.size} px x {T} frames")
    return {"value": round(pix.size * T / secs, 1), "unit": "pixel-frames/s", "cores": nthreads,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{pix.size} random pixels x {T} frames of the same clip, thresholded "
                      f"path, FP64, {secs:.1f}s; events/s {out['count'] / secs:.1f}",
            "exhaustive": {"value": round(pe.size * T / se, 1), "unit": "pixel-frames/s",
                           "sample": f"{pe.size} random pixels x {T} frames, WLR+ESIM, FP64, {se:.1f}s"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-pixels", type=int, default=640 * 480,
                    help="pixels of the clip the oracle simulates over all frames (random "
                         "sample; default all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exhaustive", action="store_true")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of a graph")
    ap.add_argument("--save-clip", type=str, default=None,
                    help="also save the generated clip (E, feat) to this file")
    ap.add_argument("--load-clip", type=str, default=None,
                    help="load the clip saved by --save-clip instead of generating it")
    ap.add_argument("--schedule", type=str, default=None,
                    help="lanes_dense,lanes_list,blocks_per_cu (skips the autotuner)")
    ap.add_argument("--workload", choices=("dvs", "precision", "batch", "diff", "quality", "threshold",
                                           "bandwidth", "multicrossing"),
                    default="dvs",
                    help="dvs (default, the contract line) or one of the extension workloads")
    ap.add_argument("--precision-frames", type=int, default=None,
                    help="frames of the precision workload (default: all 500)")
    ap.add_argument("--no-frame-log", action="store_true",
                    help="skip the per-frame record (flagged fraction, events, FP64 re-solves, "
                         "kappa-hat histogram, stuck pixels)")
    ap.add_argument("--frame-log", type=str, default=None,
                    help="write the per-frame JSON lines to this file (default: stderr)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 512 MiB read + 512 MiB write elementwise kernel (the "
                         "known-size reference for HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: sharding the clip by pixel rows across GPUs is designed "
              "but not implemented.  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2303_02608_amd import autotune
    from paper_2303_02608_amd import binding as B
    from paper_2303_02608_amd import synth
    from paper_2303_02608_amd.simulator import Simulator

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    B.load()   # raises if libesim.so is missing: there is no fallback
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload != "dvs":
        fn = {"precision": workload_precision, "batch": workload_batch, "diff": workload_diff,
              "quality": workload_quality, "threshold": workload_threshold,
              "bandwidth": workload_bandwidth, "multicrossing": workload_multicrossing}
        res = fn[args.workload](args, B, synth, Simulator)
        res = {"metric": f"{args.workload} workload", "n_gpus": 1, "dtype": "f64",
               "data": "synthetic", **res}
        print(json.dumps(res), flush=True)
        return

    cfg = synth.config_spec(1)
    spec = cfg["spec"]
    r, tr, C = cfg["r"], cfg["tr"], cfg["C"]
    T, H, W, F = spec.T, spec.H, spec.W, spec.F
    t0 = time.time()
    if args.load_clip:
        saved = torch.load(args.load_clip, map_location=dev, weights_only=True)
        E, feat = saved["E"].contiguous(), saved["feat"].contiguous()
        assert tuple(feat.shape) == (T, F, H, W)
        log(f"loaded {W}x{H}x{T} clip from {args.load_clip}")
    else:
        clip = synth.make_clip(spec, device=dev)
        torch.cuda.synchronize()
        log(f"generated {W}x{H}x{T} spp={spec.spp} F={F} in {time.time() - t0:.1f}s")
        E, feat = clip["E"].contiguous(), clip["feat"].contiguous()
        if args.save_clip:
            torch.save({"E": E.cpu(), "feat": feat.cpu()}, args.save_clip)
    y = torch.empty_like(E)
    params = B.Params(r=r, tr=tr, C=C, dt=cfg["dt"])
    sim = Simulator(y, feat, params)
    pf = T * H * W
    B.log_brightness(E, out=y)
    t0 = time.time()
    if args.schedule:
        sched = tuple(int(v) for v in args.schedule.split(","))
        sim.plan.set_schedule(*sched)
        log(f"schedule (lanes dense, lanes list, blocks/CU) = {sched} (given)")
    else:
        sched = autotune.tune(sim.plan, verbose=False)
        log(f"autotuned schedule (lanes dense, lanes list, blocks/CU) = {sched} "
            f"in {time.time() - t0:.1f}s")

    def step(mode):
        B.log_brightness(E, out=y)
        sim.enqueue(mode)

    def timed(mode):
        if not args.eager:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                step(mode)
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                step(mode)
            run = g.replay
        else:
            run = lambda: step(mode)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) / args.steps * 1e3
        ms = e0.elapsed_time(e1) / args.steps
        ev = sim.events()
        return ms, wall, ev

    if args.copy_probe:
        a = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log("copy probe: 3 x (512 MiB read + 512 MiB write)")

    ms_thr, wall_thr, ev_thr = timed("thresholded")
    # every flagged pixel emits exactly one event, so the flagged fraction is
    # events / ((T - 1) H W)
    phi = float(ev_thr["count"]) / ((T - 1) * H * W)
    log(f"thresholded: {ms_thr:.3f} ms/step (wall {wall_thr:.3f}), events {ev_thr['count']}, "
        f"flagged fraction {phi:.4f}")
    exh = None
    if not args.no_exhaustive:
        ms_exh, wall_exh, ev_exh = timed("exhaustive")
        log(f"exhaustive: {ms_exh:.3f} ms/step (wall {wall_exh:.3f}), events {ev_exh['count']}")
        exh = dict(value=pf / (ms_exh * 1e-3), unit="pixel-frames/s", ms_per_step=ms_exh,
                   events_per_s=ev_exh["count"] / (ms_exh * 1e-3), events=ev_exh["count"])

    # ---- roofline of the regression kernel: instrumented eager pass --------
    # The thresholded path launches the regression kernel twice over: one dense
    # launch at frame 0 (lanes_dense instance) and one work-list launch per
    # later frame (lanes_list instance).  The dominant kernel is the list one.
    # The pass runs the frames as separate threshold / regress / events calls so
    # that HIP events can bracket each regression launch on its stream: the
    # same kernel instance, grid and items as inside esim_step (which only
    # differs in writing the model to the state instead of output arrays).
    stream = torch.cuda.current_stream()
    marks = []
    orig = B.regress

    def timed_regress(*a, **k):
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        orig(*a, **k)
        s1.record(stream)
        marks.append((a[2] is None, s0, s1))

    B.regress = timed_regress
    try:
        B.log_brightness(E, out=y)
        sim.enqueue("thresholded", fused=False)
        torch.cuda.synchronize()
    finally:
        B.regress = orig
    dense_ms = np.array([a.elapsed_time(b) for d, a, b in marks if d])
    list_ms = np.array([a.elapsed_time(b) for d, a, b in marks if not d])
    ev = sim.events()
    fl_dense = regress_flops(omega_sizes(np.arange(H * W) % W, np.arange(H * W) // W,
                                         np.zeros(H * W, np.int64), W, H, T, r, tr), F).sum()
    fl_list = regress_flops(omega_sizes(ev["x"].astype(np.int64), ev["y"].astype(np.int64),
                                        ev["t"].astype(np.int64), W, H, T, r, tr), F).sum()
    achieved = fl_list / (list_ms.sum() * 1e-3) / 1e12
    traffic = traffic_from_profile(None)
    ld, ll, bpc = sched
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_ALU_TFLOPS, 4),
            "traffic": traffic, "kernel": f"regress_kernel<F={F},L={ll},f32> (work-list launches)",
            "launches": int(list_ms.size), "avg_launch_ms": round(float(list_ms.mean()), 4),
            "flop_per_launch": float(fl_list / list_ms.size),
            "regress_share_of_step": round(float(list_ms.sum() + dense_ms.sum()) / ms_thr, 3),
            "dense_frame0": {"kernel": f"regress_kernel<F={F},L={ld},f32>",
                             "ms": round(float(dense_ms.sum()), 4),
                             "tflops": round(fl_dense / (dense_ms.sum() * 1e-3) / 1e12, 3)}}
    log(f"regress list launches: {list_ms.size}, avg {list_ms.mean():.4f} ms, {achieved:.2f} TFLOP/s; "
        f"dense frame 0: {dense_ms.sum():.3f} ms")
    # End to end: the time the step would take at the bounding roofline of each
    # part -- regression FLOPs at the FP64 issue peak, plus the HBM-bound
    # steps' algorithmic bytes at 8 TB/s (log 8 B per pixel-frame; threshold
    # 3F*4 + 4 B per pixel-frame t >= 1; compaction 8 B work list + 13 B event
    # per flagged pixel) -- divided by the measured step.
    flops = fl_dense + fl_list
    hbm = 8.0 * T * H * W + (3 * F * 4 + 4) * (T - 1) * H * W + 21.0 * ev["count"]
    bound_ms = (flops / (PEAK_ALU_TFLOPS * 1e12) + hbm / (PEAK_HBM_GBS * 1e9)) * 1e3
    roof["end_to_end"] = {"bound_ms": round(bound_ms, 3), "measured_ms": round(ms_thr, 3),
                          "frac": round(bound_ms / ms_thr, 4),
                          "model": "regression FLOP at 78.6 TFLOP/s + HBM-bound bytes at 8 TB/s"}

    # ---- dense (exhaustive) regression roofline, same method ---------------
    if exh is not None:
        marks.clear()
        B.regress = timed_regress
        try:
            sim.enqueue("exhaustive", fused=False)
            torch.cuda.synchronize()
        finally:
            B.regress = orig
        d2 = np.array([a.elapsed_time(b) for _, a, b in marks])
        tt = np.repeat(np.arange(T, dtype=np.int64), H * W)
        om = omega_sizes(np.tile(np.arange(H * W) % W, T), np.tile(np.arange(H * W) // W, T), tt,
                         W, H, T, r, tr)
        exh["regress_tflops"] = round(regress_flops(om, F).sum() / (d2.sum() * 1e-3) / 1e12, 3)
        exh["regress_frac"] = round(exh["regress_tflops"] / PEAK_ALU_TFLOPS, 4)

    # ---- per-frame record (untimed): phi, events, re-solves, kappa-hat, stuck
    flog = None
    if not args.no_frame_log:
        fh = open(args.frame_log, "w") if args.frame_log else sys.stderr

        def emit(rec):
            print(json.dumps({"frame_log": rec}), file=fh, flush=True)

        try:
            flog = frame_log(sim, feat, params, emit)
        finally:
            if fh is not sys.stderr:
                fh.close()
        log(f"frame log: phi {flog['phi_min']}..{flog['phi_max']}, stuck pixels at the last "
            f"frame {flog['stuck_last_frame']}, kappa-hat histogram {flog['kappa_hist_decades_from_1']}")

    # ---- CPU baseline: the FP64 oracle on a random pixel sample -----------
    cpu = None if args.no_cpu_baseline else cpu_baseline(E, feat, r, tr, C, args.cpu_pixels)

    res = {
        "metric": METRIC,
        "value": round(pf / (ms_thr * 1e-3), 1),
        "unit": "pixel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_thr, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"DVS {W}x{H}x{T}, {spec.spp} spp, F={F} f32, r={r}, tr={tr}, "
                               f"C={C}, thresholded path",
                   "W": W, "H": H, "T": T, "spp": spec.spp, "F": F, "r": r, "tr": tr, "C": C,
                   "graph": not args.eager, "schedule": list(sched)},
        "events_per_s": round(ev_thr["count"] / (ms_thr * 1e-3), 1),
        "events": ev_thr["count"],
        "flagged_fraction": round(phi, 5),
        "exhaustive": exh,
        "speedup_vs_exhaustive": round(exh["ms_per_step"] / ms_thr, 3) if exh else None,
        "roofline": roof,
        "frame_log": flog,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
