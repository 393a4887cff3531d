"""GPU parity of the adjoint (esim_wlr_backward) with the FP64 oracle's
adjoint, which is itself pinned to central finite differences on the CPU."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from paper_2303_02608_amd.autograd import wlr_alpha
from parity_util import oracle_clip, say, to_dev

pytestmark = pytest.mark.gpu


def _check_backward(E, feat, r, tr, b, items, ga, ridge=1e-6, tag=""):
    T, F, H, W = feat.shape
    HW = H * W
    y, fd = to_dev(E, feat)
    y = y.clone().requires_grad_(True)
    bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
    it_dev = torch.from_numpy(((items // HW).astype(np.int64) << 44) | (items % HW)).cuda()
    alpha = wlr_alpha(y, bt, fd, it_dev, r, tr, C=0.2, ridge=ridge)
    (alpha * torch.from_numpy(ga).float().cuda()).sum().backward()
    torch.cuda.synchronize()
    gy = y.grad.cpu().numpy().astype(np.float64)
    gb = bt.grad.numpy()
    clip = oracle_clip(E, feat)
    ref_y, ref_b, fails = oracle.backward(clip, oracle.Params(r, tr, 0.2, 1.0, b, ridge), items, ga)
    assert fails == 0
    scale = max(1e-12, np.abs(ref_y).max())
    ey = np.abs(gy - ref_y).max() / scale
    eb = np.abs(gb - ref_b) / np.maximum(1e-3 * np.abs(ref_b).max(), np.abs(ref_b))
    say(f"backward {tag}: max |dgy|/max|gy| {ey:.2e}, max rel dgb {eb.max():.2e}")
    assert ey <= 1e-4
    assert eb.max() <= 1e-4
    # the forward alpha too
    th = oracle.regress_items(clip, oracle.Params(r, tr, 0.2, 1.0, b, ridge), items)["theta"][:, 0]
    a = alpha.detach().cpu().numpy()
    assert np.max(np.abs(a - th) / np.maximum(1, np.abs(th))) <= 1e-4


@pytest.mark.parametrize("F,r,tr,seed", [(3, 2, 1, 1), (7, 3, 1, 2), (1, 1, 0, 3), (10, 2, 2, 4)])
def test_backward_matches_oracle_random(F, r, tr, seed):
    say(f"backward random F={F} r={r} tr={tr}")
    T, H, W = 5, 19, 23
    d = synth.random_features_clip(W, H, T, F, seed)
    rng = np.random.default_rng(seed)
    items = np.unique(rng.integers(0, T * H * W, size=150))
    ga = rng.standard_normal(items.size)
    ga[::7] = 0.0
    b = list(rng.uniform(0.7, 1.4, size=F + 2))
    _check_backward(d["E"].numpy(), d["feat"].numpy(), r, tr, b, items, ga, tag=f"F={F}")


def test_backward_small_workload(small_clip):
    say("backward small workload")
    E, feat = small_clip["E"][:6], small_clip["feat"][:6]
    T, F, H, W = feat.shape
    rng = np.random.default_rng(7)
    items = np.unique(rng.integers(0, T * H * W, size=400))
    ga = rng.standard_normal(items.size)
    _check_backward(E, feat, 5, 1, [1.0] * (F + 2), items, ga, tag="small")


def test_backward_accumulates_and_is_deterministic(small_clip):
    E, feat = small_clip["E"][:4, :32, :32], small_clip["feat"][:4, :, :32, :32]
    T, F, H, W = feat.shape
    say("backward determinism")
    y, fd = to_dev(E, feat)
    plan = B.Plan([y], [fd], [B.Params(3, 1, 0.2)])
    rng = np.random.default_rng(1)
    items_np = np.unique(rng.integers(0, T * H * W, size=300))
    items = torch.from_numpy(((items_np // (H * W)) << 44) | (items_np % (H * W))).cuda()
    ga = torch.from_numpy(rng.standard_normal(items_np.size)).float().cuda()
    scratch = torch.empty(B.backward_scratch_bytes(plan, items.numel()), dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(2):
        gy = torch.zeros_like(y)
        gb = torch.zeros(F + 2, dtype=torch.float64, device="cuda")
        B.backward(plan, items, ga, gy, gb, scratch)
        B.backward(plan, items, ga, gy, gb, scratch)     # accumulates
        torch.cuda.synchronize()
        outs.append((gy.clone(), gb.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    gy1 = torch.zeros_like(y)
    gb1 = torch.zeros(F + 2, dtype=torch.float64, device="cuda")
    B.backward(plan, items, ga, gy1, gb1, scratch)
    torch.cuda.synchronize()
    assert torch.allclose(outs[0][0], 2 * gy1, rtol=1e-6, atol=1e-9)
    assert torch.allclose(outs[0][1], 2 * gb1, rtol=1e-12, atol=0)


def test_backward_graph_replays(small_clip):
    """esim_wlr_backward captured in a graph (after zeroing its accumulated
    outputs with fill kernels): replays, with eager work and synchronisation
    between them, give the eager gradients bit for bit."""
    E, feat = small_clip["E"][:5], small_clip["feat"][:5]
    T, F, H, W = feat.shape
    say("backward graph replays")
    y, fd = to_dev(E, feat)
    plan = B.Plan([y], [fd], [B.Params(4, 1, 0.2)])
    rng = np.random.default_rng(3)
    items_np = np.unique(rng.integers(0, T * H * W, size=500))
    items = torch.from_numpy(((items_np // (H * W)) << 44) | (items_np % (H * W))).cuda()
    ga = torch.from_numpy(rng.standard_normal(items_np.size)).float().cuda()
    scratch = torch.empty(B.backward_scratch_bytes(plan, items.numel()), dtype=torch.uint8, device="cuda")
    gy = torch.zeros_like(y)
    gb = torch.zeros(F + 2, dtype=torch.float64, device="cuda")

    def run():
        gy.zero_()
        gb.zero_()
        B.backward(plan, items, ga, gy, gb, scratch)

    run()
    torch.cuda.synchronize()
    ref_y, ref_b = gy.clone(), gb.clone()
    assert torch.count_nonzero(ref_y) > 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for _ in range(3):
        gy.fill_(1.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(gy, ref_y) and torch.equal(gb, ref_b)
        _ = (y * 2).sum().item()


@pytest.mark.parametrize("F,r,tr,W,H,seed", [(4, 9, 1, 41, 37, 6), (2, 25, 0, 83, 61, 7)])
def test_backward_wide_windows(F, r, tr, W, H, seed):
    """Windows wider than 16 columns: the item kernel runs 4 lanes per item, and
    at r = 25 a gather block's item region spans 66 columns and 66 rows (the
    widest packed positions)."""
    say(f"backward wide window F={F} r={r} tr={tr} {W}x{H}")
    T = 4
    d = synth.random_features_clip(W, H, T, F, seed)
    rng = np.random.default_rng(seed)
    items = np.unique(rng.integers(0, T * H * W, size=120))
    ga = rng.standard_normal(items.size)
    b = list(rng.uniform(0.7, 1.4, size=F + 2))
    _check_backward(d["E"].numpy(), d["feat"].numpy(), r, tr, b, items, ga, tag=f"F={F} r={r}")


@pytest.mark.parametrize("F,r,tr,seed", [(12, 3, 1, 8), (7, 4, 1, 9)])
def test_backward_dense_items(F, r, tr, seed):
    """Every pixel of every frame is an item, so a gather block's region holds
    far more items than its LDS buffer (117 items at F = 12, 179 at F = 7): the
    buffer is walked several times within one step of 256 slots, and the step
    resumes after each walk."""
    say(f"backward dense items F={F} r={r} tr={tr}")
    T, H, W = 4, 26, 37
    d = synth.random_features_clip(W, H, T, F, seed)
    rng = np.random.default_rng(seed)
    items = np.arange(T * H * W, dtype=np.int64)
    ga = rng.standard_normal(items.size)
    ga[::5] = 0.0
    b = list(rng.uniform(0.7, 1.4, size=F + 2))
    _check_backward(d["E"].numpy(), d["feat"].numpy(), r, tr, b, items, ga, tag=f"dense F={F}")
