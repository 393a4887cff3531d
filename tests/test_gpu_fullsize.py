"""Parity at the full workload sizes, in the launch configuration the benchmark
times (autotuned schedule): every pixel's event history of the DVS clip
(thresholded and raw ESIM, one event per pixel-frame and every crossing),
sampled pixels' histories where the oracle needs a regression per pixel-frame
(WLR+ESIM), whole frames of regressions, the event-set comparison, the
32-clip batch, sampled adjoint items, and finite differences of the full
differentiation loss."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import autotune
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from paper_2303_02608_amd.autograd import wlr_alpha
from paper_2303_02608_amd.simulator import Simulator
from parity_util import MODE_ID, compare_events, compare_every_crossing, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dvs():
    cfg = synth.config_spec(1)
    say("generate DVS 640x480x120 on the GPU")
    d = synth.make_clip(cfg["spec"], device="cuda")
    E, feat = d["E"], d["feat"]
    y = B.log_brightness(E)
    torch.cuda.synchronize()
    return dict(cfg=cfg, E=E, feat=feat, y=y, En=E.cpu().numpy(), fn=feat.cpu().numpy())


def _oracle_clip(d):
    if "oc" not in d:
        d["oc"] = oracle.Clip(oracle.log_brightness(d["En"]), d["fn"])
    return d["oc"]


@pytest.mark.parametrize("mode", ["thresholded", "raw"])
def test_dvs_events_whole_clip(dvs, mode):
    """Every pixel's event history of the DVS clip (launched as the benchmark
    launches it: autotuned schedule, step entry point) against the oracle's
    run over the whole clip."""
    cfg = dvs["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], dt=cfg["dt"])
    sim = Simulator(dvs["y"], dvs["feat"], p)
    sched = autotune.tune(sim.plan)
    say(f"DVS {mode} whole clip, schedule {sched}")
    gpu = sim.run(mode)
    T, F, H, W = dvs["fn"].shape
    orc = oracle.run(_oracle_clip(dvs), oracle.Params(p.r, p.tr, p.C), MODE_ID[mode], want_dl=True)
    n, exc, fails = compare_events(gpu, orc, W, p.C, 1e-4)
    say(f"DVS {mode}: {n} pixels, gpu {gpu['count']} / oracle {orc['count']} events, excused {exc}")
    assert not fails, fails[:5]
    assert exc <= n // 1000
    assert orc["count"] > 0


def test_dvs_exhaustive_events_on_sampled_pixels(dvs):
    """WLR+ESIM on the whole DVS clip against the oracle's whole histories of
    1024 pixels (512 random, 512 that fire); the oracle's every-pixel-frame
    regression makes the whole clip too slow for a test."""
    cfg = dvs["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], dt=cfg["dt"])
    sim = Simulator(dvs["y"], dvs["feat"], p)
    sched = autotune.tune(sim.plan)
    say(f"DVS exhaustive, schedule {sched}")
    gpu = sim.run("exhaustive")
    T, F, H, W = dvs["fn"].shape
    rng = np.random.default_rng(11)
    fired = np.unique(gpu["y"].astype(np.int64) * W + gpu["x"])
    pix = np.unique(np.concatenate([rng.choice(H * W, 512, replace=False),
                                    rng.choice(fired, min(512, fired.size), replace=False)]))
    orc = oracle.run(_oracle_clip(dvs), oracle.Params(p.r, p.tr, p.C), oracle.EXHAUSTIVE, pixels=pix,
                     want_dl=True)
    n, exc, fails = compare_events(gpu, orc, W, p.C, 1e-4, pixels=pix)
    say(f"DVS exhaustive: {n} sampled pixels, {orc['count']} oracle events, excused {exc}")
    assert not fails, fails[:5]
    assert exc <= 2
    assert orc["count"] > 0


def test_dvs_raw_multicrossing_whole_clip(dvs):
    """Every-crossing raw ESIM on the whole DVS clip, launched as the
    every-crossing workload launches it (the step entry point), against the
    oracle's every-crossing rule run from E on every pixel (the rule alone is
    cheap on the host)."""
    cfg = dvs["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], multi_crossing=True, dt=cfg["dt"])
    T, F, H, W = dvs["fn"].shape
    say("DVS every-crossing raw, whole clip")
    sim = Simulator(dvs["y"], dvs["feat"], p, capacity=1 << 27)
    gpu = sim.run("raw")
    assert 0 < gpu["count"] < sim.ev.capacity
    oc = _oracle_clip(dvs)
    orc = oracle.run(oc, oracle.Params(p.r, p.tr, p.C), oracle.RAW_ALL, want_dl=True)
    n, exc, fails, err = compare_every_crossing(gpu, orc, oc.y.reshape(T, H * W), W, p.C, dt=p.dt)
    say(f"DVS every-crossing raw: {n} pixels, gpu {gpu['count']} / oracle {orc['count']} events, "
        f"excused {exc}, max time error {err:.2e} frames")
    assert not fails, fails[:5]
    assert exc <= n // 1000


def test_dvs_exhaustive_multicrossing_on_sampled_pixels(dvs):
    """Every-crossing WLR+ESIM on the whole DVS clip (step entry point) against
    the oracle's every-crossing WLR+ESIM from E on sampled pixels' whole
    histories (its own FP64 regressions of every frame)."""
    cfg = dvs["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], multi_crossing=True, dt=cfg["dt"])
    T, F, H, W = dvs["fn"].shape
    HW = H * W
    say("DVS every-crossing exhaustive")
    sim = Simulator(dvs["y"], dvs["feat"], p, capacity=1 << 27)
    gpu = sim.run("exhaustive")
    assert 0 < gpu["count"] < sim.ev.capacity
    rng = np.random.default_rng(17)
    gp = gpu["y"].astype(np.int64) * W + gpu["x"]
    fired = np.unique(gp)
    pix = np.unique(np.concatenate([rng.choice(HW, 64, replace=False),
                                    rng.choice(fired, min(64, fired.size), replace=False)]))
    oc = _oracle_clip(dvs)
    op = oracle.Params(p.r, p.tr, p.C)
    orc = oracle.run(oc, op, oracle.EXHAUSTIVE_ALL, pixels=pix, want_dl=True)
    items = (np.arange(T, dtype=np.int64)[:, None] * HW + pix[None, :]).reshape(-1)
    alpha = oracle.regress_items(oc, op, items)["theta"][:, 0].reshape(T, pix.size)
    n, exc, fails, err = compare_every_crossing(gpu, orc, alpha, W, p.C, dt=p.dt, pixels=pix)
    say(f"DVS every-crossing exhaustive: {n} sampled pixels, {orc['count']} oracle events, "
        f"excused {exc}, max time error {err:.2e} frames")
    assert orc["count"] > pix.size
    assert not fails, fails[:5]
    assert exc <= 2


@pytest.mark.parametrize("form", ["last", "new"])
def test_dvs_explicit_thresholds_on_sampled_pixels(dvs, form):
    """The explicit Delta R thresholds on the whole DVS clip (the launch
    configuration of the threshold-forms workload) against the oracle's
    explicit runs on sampled pixels; band as in the small-workload test."""
    cfg = dvs["cfg"]
    thr, omode = ((B.THRESHOLD_LAST_WINDOW, oracle.EXPLICIT_LAST) if form == "last"
                  else (B.THRESHOLD_NEW_WINDOW, oracle.EXPLICIT_NEW))
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], threshold=thr)
    sim = Simulator(dvs["y"], dvs["feat"], p)
    sched = autotune.tune(sim.plan)
    say(f"DVS explicit threshold {form}, schedule {sched}")
    gpu = sim.run("thresholded")
    T, F, H, W = dvs["fn"].shape
    rng = np.random.default_rng(13)
    fired = np.unique(gpu["y"].astype(np.int64) * W + gpu["x"])
    pix = np.unique(np.concatenate([rng.choice(H * W, 48, replace=False),
                                    rng.choice(fired, min(48, fired.size), replace=False)]))
    orc = oracle.run(_oracle_clip(dvs), oracle.Params(p.r, p.tr, p.C), omode, pixels=pix, want_dl=True)
    n, exc, fails = compare_events(gpu, orc, W, p.C, 1e-3, pixels=pix)
    say(f"DVS explicit {form}: {n} sampled pixels, {orc['count']} oracle events, excused {exc}")
    assert not fails, fails[:5]
    assert exc <= 2
    assert orc["count"] > 0


def test_dvs_bandwidth_regression_on_sampled_pixels():
    """The bandwidth-optimised regression on a frame of the DVS clip (dense
    launch, as the bandwidth workload runs it) against the oracle on sampled
    pixels; the choice band as in the small-workload test."""
    cfg = synth.config_spec(1)
    say("DVS bandwidth regression, frame 57")
    d = synth.make_clip(cfg["spec"], device="cuda", frames=range(55, 60))
    E, var, feat = d["E"], d["var"], d["feat"]
    y = B.log_brightness(E)
    vy = B.log_variance(E, var, cfg["spec"].spp)
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"])
    plan = B.Plan([y], [feat], [p])
    HW = plan.npix
    hs = [0.5, 0.75, 1.0, 1.5, 2.0]
    a = torch.empty(HW, device="cuda")
    h = torch.empty(HW, device="cuda")
    s = torch.empty(HW, device="cuda")
    B.regress_bandwidth(plan, 2, None, None, HW, vy, hs, a, None, h, s)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    pix = rng.choice(HW, 300, replace=False)
    En, vn = E.cpu().numpy(), var.cpu().numpy()
    oc = oracle.Clip(oracle.log_brightness(En), feat.cpu().numpy())
    o = oracle.regress_bandwidth(oc, oracle.Params(p.r, p.tr, p.C), np.array(hs),
                                 oracle.log_variance(En, vn, cfg["spec"].spp), 2 * HW + pix)
    hg = h.cpu().numpy()[pix]
    kg = np.searchsorted(np.array(hs), hg)
    rows = np.arange(pix.size)
    sm = o["sure"].min(axis=1)
    so = o["sure"][rows, kg]
    flips = int(np.sum(kg != np.argmin(o["sure"], axis=1)))
    say(f"DVS bandwidth: {flips} of {pix.size} choices differ from the oracle's")
    assert np.all(so - sm <= 1e-5 + 1e-4 * np.abs(sm))
    assert flips <= 3
    ao = o["alpha_k"][rows, kg]
    assert np.max(np.abs(a.cpu().numpy()[pix] - ao) / np.maximum(1, np.abs(ao))) <= 1e-4


def test_dvs_event_quality():
    """The event-set comparison on the quality workload's full sets: the
    thresholded conversion of the DVS clip against ESIM on its noise-free
    frames, GPU precision, recall and Chamfer distance equal to the oracle's
    (k-d tree per polarity) over all events; and raw ESIM's 28 M noisy events,
    whose GPU nearest-neighbour distances are checked on a sample of queries."""
    from oracle import metrics as OM
    from paper_2303_02608_amd import quality as Q
    cfg = synth.config_spec(1)
    say("generate DVS 640x480x120 with reference frames")
    d = synth.make_clip(cfg["spec"], device="cuda", reference=True)
    feat = d["feat"]
    T, F, H, W = feat.shape
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"])
    ref = Simulator(B.log_brightness(d["E_ref"]), feat, p).run("raw")
    y = B.log_brightness(d["E"])
    taus, rmax = [5e-4, 2e-3, 5e-3, 1e-2], 0.05
    keys = ("x", "y", "t", "p")
    r = {k: ref[k] for k in keys}
    gen = Simulator(y, feat, p).run("thresholded")
    g = {k: gen[k] for k in keys}
    m = Q.metrics(Q.to_device(g), Q.to_device(r), W, H, T, taus, rmax)
    o = OM.metrics(g, r, W, H, T, taus, rmax)
    say(f"DVS thresholded vs reference: {gen['count']} / {ref['count']} events, F {m['F']}")
    assert m["P"] == pytest.approx(o["P"], rel=1e-12) and m["R"] == pytest.approx(o["R"], rel=1e-12)
    assert m["CD"] == pytest.approx(o["CD"], rel=1e-12)
    raw = Simulator(y, feat, p, capacity=1 << 26).run("raw")
    assert raw["count"] < 1 << 26
    q = {k: raw[k] for k in keys}
    dist = B.nn_distances(Q.to_device(r), Q.to_device(q), W, H, T, rmax).cpu().numpy()
    assert dist.size == raw["count"]
    sel = np.random.default_rng(23).choice(raw["count"], 50000, replace=False)
    od = OM.nn_distances(r, {k: v[sel] for k, v in q.items()}, W, H, T, rmax)
    say(f"DVS raw: {raw['count']} queries, {sel.size} checked, {np.isfinite(od).mean():.3f} within rmax")
    ds = dist[sel]
    # a lattice offset of exactly rmax (32 columns, 24 rows or 6 frames at
    # rmax = 0.05) is rounded to either side of rmax: the GPU scales integer
    # offsets, the oracle subtracts scaled coordinates.  Such a distance is
    # finite on one side and +inf on the other; elsewhere the two agree.
    edge = (np.abs(ds - rmax) <= 1e-12 * rmax) | (np.abs(od - rmax) <= 1e-12 * rmax)
    say(f"DVS raw: {int(edge.sum())} distances at rmax up to rounding")
    assert np.array_equal(np.isinf(ds[~edge]), np.isinf(od[~edge]))
    f = np.isfinite(od) & np.isfinite(ds)
    assert np.allclose(ds[f], od[f], rtol=1e-12, atol=0)
    assert np.all(np.isfinite(ds[edge]) | np.isfinite(od[edge]))


def test_dvs_regressions_full_frames(dvs):
    """Dense regressions of whole DVS frames (first, middle, last) against the
    oracle at every pixel: alpha and beta to 1e-4 relative."""
    cfg = dvs["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"])
    plan = B.Plan([dvs["y"]], [dvs["feat"]], [p])
    HW = plan.npix
    a = torch.empty(HW, device="cuda")
    b = torch.empty((plan.D, HW), device="cuda")
    for t in (0, 57, 119):
        say(f"DVS dense regression t={t}, every pixel")
        B.regress(plan, t, None, None, HW, a, b)
        torch.cuda.synchronize()
        ref = oracle.regress_items(_oracle_clip(dvs), oracle.Params(p.r, p.tr, p.C),
                                   t * HW + np.arange(HW, dtype=np.int64))
        th = ref["theta"]
        ea = np.abs(a.cpu().numpy() - th[:, 0]) / np.maximum(1, np.abs(th[:, 0]))
        eb = np.abs(b.cpu().numpy().T - th[:, 1:]) / np.maximum(1, np.abs(th[:, 1:]))
        say(f"t={t}: {HW} pixels, alpha {ea.max():.2e} beta {eb.max():.2e}")
        assert ref["fails"] == 0
        assert ea.max() <= 1e-4 and eb.max() <= 1e-4


def test_batch_workload():
    """The 32-clip batch (per-clip flagged fractions aimed at 1-40 %; frames
    scaled to 4e8 pixel-frames for the test budget, the benchmark runs every
    clip at full length), launched as the benchmark launches it: each clip's
    batched events equal its own conversion, the three smallest clips match
    the oracle at every pixel, and sampled pixels of four more (the largest
    frame, the widest radius, the longest and the smallest frame) over their
    whole histories."""
    from paper_2303_02608_amd.simulator import BatchSimulator
    specs = synth.batch_specs(32, seed=5000, max_pixel_frames=4e8)
    area = [c["spec"].W * c["spec"].H for c in specs]
    vol = [a * c["spec"].T for a, c in zip(area, specs)]
    whole = [int(k) for k in np.argsort(vol)[:3]]
    pick = sorted({int(np.argmax(area)), int(np.argmax([c["r"] for c in specs])),
                   int(np.argmax([c["spec"].T for c in specs])), int(np.argmin(area))} - set(whole))
    say(f"generate the 32-clip batch; oracle on every pixel of clips {whole}, sampled on {pick}")
    ys, feats, params, host = [], [], [], {}
    for i, c in enumerate(specs):
        d = synth.make_clip(c["spec"], device="cuda")
        ys.append(B.log_brightness(d["E"]))
        feats.append(d["feat"])
        params.append(B.Params(r=c["r"], tr=c["tr"], C=c["C"], dt=c["dt"]))
        if i in pick or i in whole:
            host[i] = (d["E"].cpu().numpy(), d["feat"].cpu().numpy())
        del d
    bs = BatchSimulator(ys, feats, params)
    got = bs.run()
    say(f"batch: {got['count']} events")
    assert 0 < got["count"] < bs.ev.capacity
    for c in range(len(specs)):
        m = got["clip"] == c
        single = Simulator(ys[c], feats[c], params[c]).run("thresholded")
        for k in ("x", "y", "t", "p"):
            assert np.array_equal(got[k][m], single[k]), (c, k)
    rng = np.random.default_rng(29)
    for c in whole + pick:
        E, feat = host[c]
        T, F, H, W = feat.shape
        p = params[c]
        m = got["clip"] == c
        g = {k: got[k][m] for k in ("x", "y", "t", "p")}
        if c in whole:
            pix = None
        else:
            fired = np.unique(g["y"].astype(np.int64) * W + g["x"])
            pix = np.unique(np.concatenate([rng.choice(H * W, 24, replace=False),
                                            rng.choice(fired, min(24, fired.size), replace=False)]))
        orc = oracle.run(oracle.Clip(oracle.log_brightness(E), feat), oracle.Params(p.r, p.tr, p.C),
                         oracle.THRESHOLDED, pixels=pix, want_dl=True)
        n, exc, fails = compare_events(g, orc, W, p.C, 1e-4, pixels=pix)
        say(f"clip {c} ({W}x{H}x{T}, r={p.r}): {n} pixels, {orc['count']} oracle events, excused {exc}")
        assert not fails, (c, fails[:5])
        assert exc <= max(2, n // 1000)


@pytest.fixture(scope="module")
def diff_clip():
    cfg = synth.config_spec(3)
    say("generate differentiation clip 640x480x60 on the GPU")
    d = synth.make_clip(cfg["spec"], device="cuda")
    y = B.log_brightness(d["E"])
    torch.cuda.synchronize()
    return dict(cfg=cfg, E=d["E"], feat=d["feat"], y=y)


def _loss_items(dc):
    """Items of the differentiation loss: every regression of the thresholded
    forward pass (all pixels at frame 0, then one per event), with, for each
    event, the index of the same pixel's previous regression."""
    cfg = dc["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"])
    ev = Simulator(dc["y"], dc["feat"], p).run("thresholded")
    T, F, H, W = dc["feat"].shape
    HW = H * W
    pix_ev = ev["y"].astype(np.int64) * W + ev["x"]
    t_ev = ev["t"].astype(np.int64)
    items = np.concatenate([np.arange(HW, dtype=np.int64), (t_ev << 44) | pix_ev])
    last = np.arange(HW, dtype=np.int64)          # index of each pixel's latest regression
    prev = np.empty(pix_ev.size, np.int64)
    for k, q in enumerate(pix_ev):                # events are in (t, py, px) order
        prev[k] = last[q]
        last[q] = HW + k
    return items, prev, p


def _loss(alpha, prev, HW):
    d = alpha[HW:] - alpha[torch.from_numpy(prev).cuda()]
    return (d.double() ** 2).sum()


def test_diff_loss_gradient_full_size(diff_clip):
    """Full differentiation loss sum over flagged regressions of
    (alpha_t - alpha_ref)^2 with the flag set frozen: the adjoint's gradient
    against central finite differences of the same GPU forward, for all seven
    buffer bandwidths and the two coordinate bandwidths (h = 1e-3) and for 64
    sampled brightness entries.  alpha is linear in y (the weights depend on
    the features only), so the loss is quadratic in each y entry and its
    central difference is exact for any step: the y step is 0.5, large enough
    that the FP32 outputs of the forward pass resolve it."""
    dc = diff_clip
    items, prev, p = _loss_items(dc)
    T, F, H, W = dc["feat"].shape
    HW = H * W
    say(f"diff loss: {items.size} regressions")
    it = torch.from_numpy(items).cuda()
    b = torch.ones(F + 2, dtype=torch.float64, requires_grad=True)
    y = dc["y"].clone().requires_grad_(True)
    alpha = wlr_alpha(y, b, dc["feat"], it, p.r, p.tr, C=p.C)
    loss = _loss(alpha, prev, HW)
    loss.backward()
    g = b.grad.numpy()
    gy = y.grad.cpu().numpy()
    assert np.all(np.isfinite(g)) and np.isfinite(gy).all()
    L0 = abs(loss.detach().item())
    h = 1e-3
    for j in range(F + 2):
        vals = []
        for sgn in (1, -1):
            bb = torch.ones_like(b).detach()
            bb[j] += sgn * h
            a2 = wlr_alpha(dc["y"], bb, dc["feat"], it, p.r, p.tr, C=p.C)
            vals.append(float(_loss(a2, prev, HW)))
        fd = (vals[0] - vals[1]) / (2 * h)
        say(f"dL/db_{j}: adjoint {g[j]:.6e} central FD {fd:.6e}")
        assert g[j] == pytest.approx(fd, rel=2e-3, abs=1e-6 * L0)
    # brightness entries: half where the gradient is largest, half at random
    rng = np.random.default_rng(31)
    flat = np.abs(gy).reshape(-1)
    top = np.argsort(flat)[-32:]
    rnd = rng.choice(np.nonzero(flat > 0)[0], 32, replace=False)
    sel = np.unique(np.concatenate([top, rnd]))
    hy = 0.5
    yd = dc["y"].detach().clone()
    yflat = yd.view(-1)
    worst = 0.0
    for q in sel:
        vals = []
        for sgn in (1, -1):
            keep = float(yflat[q])
            yflat[q] = keep + sgn * hy
            a2 = wlr_alpha(yd, torch.ones(F + 2, dtype=torch.float64), dc["feat"], it, p.r, p.tr, C=p.C)
            vals.append(float(_loss(a2, prev, HW)))
            yflat[q] = keep
        fd = (vals[0] - vals[1]) / (2 * hy)
        ad = float(gy.reshape(-1)[q])
        err = abs(ad - fd) / max(abs(fd), 1e-9 * L0)
        worst = max(worst, err)
        assert ad == pytest.approx(fd, rel=2e-3, abs=1e-7 * L0), (int(q), ad, fd)
    say(f"dL/dy at {sel.size} entries: max relative difference {worst:.2e}")


def test_diff_sampled_adjoint_items(diff_clip):
    """The adjoint at full size with the upstream gradient on a sample of the
    loss's regressions only, against the oracle's adjoint of those items."""
    dc = diff_clip
    items, prev, p = _loss_items(dc)
    rng = np.random.default_rng(5)
    sel = rng.choice(items.size, 24, replace=False)
    ga = np.zeros(items.size)
    ga[sel] = rng.standard_normal(sel.size)
    T, F, H, W = dc["feat"].shape
    HW = H * W
    y = dc["y"].clone().requires_grad_(True)
    b = torch.ones(F + 2, dtype=torch.float64, requires_grad=True)
    alpha = wlr_alpha(y, b, dc["feat"], torch.from_numpy(items).cuda(), p.r, p.tr, C=p.C)
    (alpha * torch.from_numpy(ga).float().cuda()).sum().backward()
    torch.cuda.synchronize()
    En, fn = dc["E"].cpu().numpy(), dc["feat"].cpu().numpy()
    clip = oracle.Clip(oracle.log_brightness(En), fn)
    flat = (items[sel] >> 44) * HW + (items[sel] & 0xFFFFFFFF)
    ref_y, ref_b, fails = oracle.backward(clip, oracle.Params(p.r, p.tr, p.C), flat, ga[sel])
    assert fails == 0
    gy = y.grad.cpu().numpy()
    nz = np.nonzero(ref_y)
    ey = np.abs(gy[nz] - ref_y[nz]).max() / np.abs(ref_y).max()
    eb = np.abs(b.grad.numpy() - ref_b).max() / np.abs(ref_b).max()
    say(f"sampled adjoint: g_y {ey:.2e}, g_b {eb:.2e}")
    assert ey <= 1e-4 and eb <= 1e-4
    # nothing outside the sampled items' windows
    mask = np.ones_like(gy, bool)
    mask[nz] = False
    assert np.abs(gy[mask]).max() <= 1e-6 * np.abs(ref_y).max()


def test_precision_workload_errors():
    """X1 at the precision workload's shape (1920x1080, F = 10 FP16 features,
    r = 10, tr = 2): regressions at the first, middle and last frames of the
    500 (each generated with its +-2 frame window, which is all a regression
    there reads) against the FP64 oracle at 256 sampled pixels each, per
    output: the FP64 Gram (contract path) within 1e-4 on the FP16 values, the
    compensated FP32 Gram with FP64 re-solves above the equilibrated
    condition bound 1e6 within its stated bounds; the share of re-solves over
    every pixel of those frames; the storage error of FP16 features against
    the oracle on the FP32 features."""
    import copy
    cfg = synth.config_spec(4)
    spec = cfg["spec"]
    spec32 = copy.deepcopy(spec)
    spec32.feat_dtype = "f32"
    HW = spec.W * spec.H
    rng = np.random.default_rng(8)
    rows = {}
    for tf in (2, spec.T // 2, spec.T - 3):
        say(f"precision workload: frames {tf - 2}..{tf + 2}")
        d = synth.make_clip(spec, device="cuda", frames=range(tf - 2, tf + 3))
        d32 = synth.make_clip(spec32, device="cuda", frames=range(tf - 2, tf + 3))
        y = B.log_brightness(d["E"])
        feat = d["feat"]
        assert feat.dtype == torch.float16
        En = d["E"].cpu().numpy()
        clip16 = oracle.Clip(oracle.log_brightness(En), feat.cpu().numpy())
        clip32 = oracle.Clip(oracle.log_brightness(En), d32["feat"].cpu().numpy())
        pix = rng.choice(HW, 256, replace=False)
        op = oracle.Params(cfg["r"], cfg["tr"], cfg["C"])
        ref = oracle.regress_items(clip16, op, 2 * HW + pix)
        ref32 = oracle.regress_items(clip32, op, 2 * HW + pix)
        th, th32 = ref["theta"], ref32["theta"]
        for prec in (B.GRAM_F64, B.GRAM_F32C):
            p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], precision=prec, kappa_fp64=1e6)
            plan = B.Plan([y], [feat], [p])
            a = torch.empty(HW, device="cuda")
            b = torch.empty((plan.D, HW), device="cuda")
            R = torch.empty(HW, device="cuda")
            K = torch.empty(HW, device="cuda")
            B.regress(plan, 2, None, None, HW, a, b, R, K)
            torch.cuda.synchronize()
            an, bn, Rn, Kn = a.cpu().numpy(), b.cpu().numpy(), R.cpu().numpy(), K.cpu().numpy()
            ea = np.abs(an[pix] - th[:, 0]) / np.maximum(1, np.abs(th[:, 0]))
            eb = np.abs(bn[:, pix].T - th[:, 1:]) / np.maximum(1, np.abs(th[:, 1:]))
            er = np.abs(Rn[pix] - ref["R"])
            es = np.abs(an[pix] - th32[:, 0]) / np.maximum(1, np.abs(th32[:, 0]))
            share = float(np.mean(~(Kn <= 1e6)))
            tag = "fp64" if prec == B.GRAM_F64 else "f32c"
            rows[(tf, tag)] = (ea.max(), eb.max(), er.max(), share, es.max())
            say(f"t={tf} {tag}: alpha max {ea.max():.2e} p99 {np.quantile(ea, 0.99):.2e}, beta max {eb.max():.2e}, "
                f"R max {er.max():.2e}, kappa-hat > 1e6 at {share:.4%} of pixels, "
                f"FP16 storage alpha error max {es.max():.2e} median {np.median(es):.2e}")
            if prec == B.GRAM_F64:
                assert ea.max() <= 1e-4 and eb.max() <= 1e-4
            else:
                assert ea.max() <= 2e-3 and np.quantile(ea, 0.99) <= 2e-4
            del plan
        del d, d32
