"""Bandwidth-optimised regression (per-item h from candidates by SURE with the
MC variance) on the GPU against the oracle.

Tolerances: alpha and beta of the chosen candidate as for every regression
(1e-4 max(1, |.|)).  The choice itself is an argmin over SURE values that the
two sides compute from the same definition in different precision (FP32
weights and variance input on the GPU): where the GPU takes another candidate
than the oracle, the oracle's own SURE at the GPU's choice must lie within
1e-5 + 1e-4 |SURE_min| of its minimum (an alpha error delta moves SURE by
about 2 |alpha - y_c| delta), and such flips must stay rare."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from parity_util import say

pytestmark = pytest.mark.gpu

HS = [0.5, 0.75, 1.0, 1.5, 2.0]


@pytest.fixture(scope="module")
def clip():
    cfg = synth.config_spec(0)
    d = synth.make_clip(cfg["spec"])
    return dict(cfg=cfg, E=d["E"].numpy(), var=d["var"].numpy(), feat=d["feat"].numpy(),
                spp=cfg["spec"].spp)


def _gpu(clip, p, t, items=None, hs=HS):
    E = torch.from_numpy(clip["E"]).cuda()
    var = torch.from_numpy(clip["var"]).cuda()
    feat = torch.from_numpy(clip["feat"]).cuda()
    y = B.log_brightness(E)
    vy = B.log_variance(E, var, clip["spp"])
    plan = B.Plan([y], [feat], [p])
    T, F, H, W = feat.shape
    n = H * W if items is None else len(items)
    a = torch.empty(n, device="cuda")
    b = torch.empty((F + 2, n), device="cuda")
    h = torch.empty(n, device="cuda")
    s = torch.empty(n, device="cuda")
    if items is None:
        B.regress_bandwidth(plan, t, None, None, n, vy, hs, a, b, h, s)
    else:
        wl = torch.from_numpy(np.asarray(items, np.int64)).cuda()
        cnt = torch.tensor([n, n], dtype=torch.int32, device="cuda")
        B.regress_bandwidth(plan, t, wl, cnt, n, vy, hs, a, b, h, s)
    torch.cuda.synchronize()
    return dict(alpha=a.cpu().numpy(), beta=b.cpu().numpy(), h=h.cpu().numpy(), sure=s.cpu().numpy(),
                vy=vy.cpu().numpy(), plan=plan, y=y, feat=feat)


def _oracle(clip, p, t, pix, hs=HS):
    oc = oracle.Clip(oracle.log_brightness(clip["E"]), clip["feat"])
    vy = oracle.log_variance(clip["E"], clip["var"], clip["spp"])
    T, F, H, W = clip["feat"].shape
    return oracle.regress_bandwidth(oc, oracle.Params(p.r, p.tr, p.C, p.h, p.b, p.ridge), np.asarray(hs),
                                    vy, t * H * W + np.asarray(pix, np.int64)), vy


def _compare(g, o, pix, hs=HS):
    hs = np.asarray(hs)
    # the GPU reports h in FP32: the nearest candidate, within FP32 rounding
    kg = np.argmin(np.abs(hs[None, :] - g["h"].astype(np.float64)[:, None]), axis=1)
    assert np.all(np.abs(hs[kg] - g["h"]) <= 1e-6 * hs[kg]), "the GPU's h is a candidate"
    sm = o["sure"].min(axis=1)
    rows = np.arange(len(pix))
    so = o["sure"][rows, kg]
    flips = kg != np.argmin(o["sure"], axis=1)
    assert np.all(so - sm <= 1e-5 + 1e-4 * np.abs(sm)), np.max(so - sm)
    assert flips.mean() <= 0.01, flips.mean()
    # alpha and SURE of the GPU's choice against the oracle's same candidate
    ao = o["alpha_k"][rows, kg]
    assert np.max(np.abs(g["alpha"] - ao) / np.maximum(1, np.abs(ao))) <= 1e-4
    assert np.max(np.abs(g["sure"] - so) / np.maximum(1e-3, np.abs(so))) <= 1e-3
    # beta where the choices agree (the oracle only reports the chosen theta)
    same = ~flips
    bo = o["theta"][same, 1:]
    bg = g["beta"].T[same]
    assert np.max(np.abs(bg - bo) / np.maximum(1, np.abs(bo))) <= 1e-4
    return flips.sum()


def test_log_variance_matches_oracle(clip):
    say("log variance")
    E = torch.from_numpy(clip["E"]).cuda()
    var = torch.from_numpy(clip["var"]).cuda()
    vy = B.log_variance(E, var, clip["spp"]).cpu().numpy()
    ref = oracle.log_variance(clip["E"], clip["var"], clip["spp"])
    assert np.allclose(vy, ref, rtol=2e-6, atol=0)


@pytest.mark.parametrize("t,tr", [(0, 0), (7, 1), (15, 1)])
def test_dense_bandwidth_regression_matches_oracle(clip, t, tr):
    cfg = clip["cfg"]
    p = B.Params(r=cfg["r"], tr=tr, C=cfg["C"])
    say(f"dense bandwidth regression t={t} tr={tr}")
    g = _gpu(clip, p, t)
    H, W = clip["feat"].shape[2:]
    pix = np.arange(H * W)
    o, _ = _oracle(clip, p, t, pix)
    nflip = _compare(g, o, pix)
    share = [float(np.mean(g["h"] == h)) for h in HS]
    say(f"t={t}: chosen-h shares {share}, choices differing from the oracle {nflip}")
    assert max(share) < 1.0          # the choice varies over the image


@pytest.mark.parametrize("r", [5, 8])
def test_work_list_matches_oracle_and_dense(clip, r):
    """Work lists run 16 lanes per item (one column each at r = 5; two column
    passes at r = 8): parity with the oracle, and the dense launch's results
    at the same pixels to summation-order rounding."""
    cfg = clip["cfg"]
    p = B.Params(r=r, tr=1, C=cfg["C"])
    say(f"bandwidth regression: work list r={r}")
    H, W = clip["feat"].shape[2:]
    rng = np.random.default_rng(2)
    pix = np.sort(rng.choice(H * W, 700, replace=False))
    g = _gpu(clip, p, 5, items=pix)
    o, _ = _oracle(clip, p, 5, pix)
    nflip = _compare(g, o, pix)
    d = _gpu(clip, p, 5)
    same = g["h"] == d["h"][pix]
    say(f"r={r}: {nflip} choices differ from the oracle, {np.sum(~same)} from the dense launch")
    assert np.mean(same) >= 0.99
    assert np.allclose(g["alpha"][same], d["alpha"][pix][same], rtol=1e-5, atol=1e-5)


def test_single_candidate_is_the_plain_regression(clip):
    """With the plan's own h as the only candidate, the outputs are those of
    the ordinary regression."""
    cfg = clip["cfg"]
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    say("bandwidth regression with one candidate")
    g = _gpu(clip, p, 3, hs=[1.0])
    H, W = clip["feat"].shape[2:]
    a = torch.empty(H * W, device="cuda")
    b = torch.empty((clip["feat"].shape[1] + 2, H * W), device="cuda")
    B.regress(g["plan"], 3, None, None, H * W, a, b)
    torch.cuda.synchronize()
    assert np.all(g["h"] == 1.0)
    assert np.allclose(g["alpha"], a.cpu().numpy(), rtol=1e-6, atol=1e-6)
    assert np.allclose(g["beta"], b.cpu().numpy(), rtol=1e-5, atol=1e-5)


def test_bandwidth_validation(clip):
    cfg = clip["cfg"]
    p = B.Params(r=cfg["r"], tr=0, C=cfg["C"])
    say("bandwidth regression validation")
    g = _gpu(clip, p, 0, hs=[1.0])
    vy = torch.from_numpy(g["vy"]).cuda()
    H, W = clip["feat"].shape[2:]
    a = torch.empty(H * W, device="cuda")
    for hs in ([], [1.0] * 9, [1.0, 0.0], [1.0, float("inf")]):
        with pytest.raises(B.EsimError):
            B.regress_bandwidth(g["plan"], 0, None, None, H * W, vy, hs, a)
    with pytest.raises(B.EsimError):
        B.regress_bandwidth(g["plan"], clip["feat"].shape[0], None, None, H * W, vy, [1.0], a)
    two = B.Plan([g["y"], g["y"]], [g["feat"], g["feat"]], [p, p])
    with pytest.raises(B.EsimError):
        B.regress_bandwidth(two, 0, None, None, 2 * H * W, vy, [1.0], torch.empty(2 * H * W, device="cuda"))


@pytest.mark.parametrize("F,feat_dtype,r", [(1, "f32", 4), (12, "f32", 3), (7, "f16", 5)])
def test_bandwidth_feature_counts_and_f16(F, feat_dtype, r):
    """Other instances: the extreme feature counts and FP16 features (the
    oracle decodes the same FP16 bits), dense and work list."""
    W, H, T = 40, 36, 4
    d = synth.random_features_clip(W, H, T, F, seed=80 + F, feat_dtype=feat_dtype)
    rng = np.random.default_rng(F)
    var = (d["E"].numpy() ** 2 * rng.uniform(0.2, 2.0, size=(T, H, W))).astype(np.float32)
    clip = dict(E=d["E"].numpy(), var=var, feat=d["feat"].numpy(), spp=4)
    p = B.Params(r=r, tr=1, C=0.1)
    say(f"bandwidth regression F={F} {feat_dtype} r={r}")
    pix = np.arange(H * W)
    g = _gpu(clip, p, 2)
    o, _ = _oracle(clip, p, 2, pix)
    _compare(g, o, pix)
    sel = np.sort(rng.choice(H * W, 300, replace=False))
    gl = _gpu(clip, p, 2, items=sel)
    ol, _ = _oracle(clip, p, 2, sel)
    _compare(gl, ol, sel)


def test_eight_candidates(clip):
    """The largest candidate set (8 bandwidths, unsorted)."""
    cfg = clip["cfg"]
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    hs = [1.0, 0.4, 2.5, 0.7, 1.8, 0.55, 1.25, 3.2]
    say("bandwidth regression with 8 candidates")
    g = _gpu(clip, p, 4, hs=hs)
    H, W = clip["feat"].shape[2:]
    pix = np.arange(H * W)
    o, _ = _oracle(clip, p, 4, pix, hs=hs)
    order = np.argsort(hs)
    hs_sorted = np.asarray(hs)[order]
    o_sorted = dict(o, sure=o["sure"][:, order], alpha_k=o["alpha_k"][:, order])
    _compare(g, o_sorted, pix, hs=hs_sorted)


def test_bandwidth_conversion_graph_replays(clip):
    """The thresholded conversion with the bandwidth chosen per regression (as
    the bandwidth workload captures it): graph replays, with eager work and
    synchronisation between them, reproduce the eager run's events bit for bit."""
    from paper_2303_02608_amd.simulator import Simulator
    cfg = clip["cfg"]
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    say("bandwidth conversion: graph replays")
    E = torch.from_numpy(clip["E"]).cuda()
    feat = torch.from_numpy(clip["feat"]).cuda()
    y = B.log_brightness(E)
    vy = B.log_variance(E, torch.from_numpy(clip["var"]).cuda(), clip["spp"])
    T, F, H, W = feat.shape
    sim = Simulator(y, feat, p)
    plan, n = sim.plan, H * W

    def convert():
        sim.ev.count.zero_()
        B.regress_bandwidth(plan, 0, None, None, n, vy, HS, sim.alpha, sim.beta)
        B.events(plan, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=n)
        for t in range(1, T):
            B.threshold(plan, t, sim.dl, sim.worklist, sim.count)
            B.regress_bandwidth(plan, t, sim.worklist, sim.count, n, vy, HS, sim.alpha, sim.beta)
            B.events(plan, t, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count, dl=sim.dl,
                     alpha=sim.alpha, beta=sim.beta, n_out=n)

    convert()
    torch.cuda.synchronize()
    eager = sim.events()
    assert eager["count"] > 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        convert()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        convert()
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = sim.events()
        for k in ("x", "y", "t", "p"):
            assert np.array_equal(got[k], eager[k]), k
        _ = (y * 2).sum().item()
