"""GPU nearest-neighbour distances and event-set metrics (Sec. 3, quantitative
comparison) against the oracle's (scipy k-d tree per polarity)."""
import numpy as np
import pytest
import torch

from oracle import metrics as OM
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import quality as Q
from paper_2303_02608_amd import synth
from paper_2303_02608_amd.simulator import Simulator
from parity_util import say, to_dev

pytestmark = pytest.mark.gpu


def _random_set(n, W, H, T, seed, outside=0):
    rng = np.random.default_rng(seed)
    ev = dict(x=rng.integers(0, W, n), y=rng.integers(0, H, n), t=rng.integers(0, T, n),
              p=rng.choice([-1, 1], n))
    if outside:
        ev["x"][:outside] = W + 3          # ignored as sources, +inf as queries
        ev["p"][outside:2 * outside] = 0
    return ev


@pytest.mark.parametrize("W,H,T,n,rmax,seed", [
    (64, 48, 10, 3000, 0.05, 1),
    (100, 37, 7, 800, 0.2, 2),      # W not a multiple of 32, radius over several words
    (640, 480, 120, 20000, 0.02, 3),
    (33, 5, 3, 50, 1.0, 4),         # sparse, everything in range
])
def test_nn_distances_match_oracle(W, H, T, n, rmax, seed):
    say(f"nn distances {W}x{H}x{T} n={n} rmax={rmax}")
    src = _random_set(n, W, H, T, seed, outside=5)
    qry = _random_set(n + 17, W, H, T, seed + 100, outside=3)
    d = B.nn_distances(Q.to_device(src), Q.to_device(qry), W, H, T, rmax).cpu().numpy()
    valid = (src["x"] < W) & (src["p"] != 0)
    ref = OM.nn_distances({k: v[valid] for k, v in src.items()}, qry, W, H, T, rmax)
    inq = (qry["x"] < W) & (qry["p"] != 0)
    ref[~inq] = np.inf
    assert np.array_equal(np.isinf(d), np.isinf(ref))
    f = np.isfinite(ref)
    assert np.allclose(d[f], ref[f], rtol=1e-12, atol=0)


def test_metrics_on_the_small_workload(small_clip):
    """Events of the three conversions against ESIM on the noise-free frames:
    the GPU metrics equal the oracle's on the same event sets."""
    cfg = small_clip["cfg"]
    d = synth.make_clip(cfg["spec"], reference=True)
    E, Eref, feat = d["E"].numpy(), d["E_ref"].numpy(), d["feat"].numpy()
    T, F, H, W = feat.shape
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"])
    yr, fd = to_dev(Eref, feat)
    ref = Simulator(yr, fd, p).run("raw")
    y, fd = to_dev(E, feat)
    taus, rmax = [5e-4, 1e-2, 3e-2], 0.1
    for mode in ("raw", "exhaustive", "thresholded"):
        gen = Simulator(y, fd, p).run(mode)
        g = {k: gen[k] for k in ("x", "y", "t", "p")}
        r = {k: ref[k] for k in ("x", "y", "t", "p")}
        m = Q.metrics(Q.to_device(g), Q.to_device(r), W, H, T, taus, rmax)
        o = OM.metrics(g, r, W, H, T, taus, rmax)
        say(f"{mode}: F {m['F']} CD {m['CD']:.3e}")
        assert m["P"] == pytest.approx(o["P"], rel=1e-12) and m["R"] == pytest.approx(o["R"], rel=1e-12)
        assert m["CD"] == pytest.approx(o["CD"], rel=1e-12)


def test_nn_distances_in_a_graph():
    """esim_nn_distances captured in a graph (the bitmap clear is a fill kernel):
    replays after the source events change in place give the eager distances
    of the new events, bit for bit."""
    W, H, T, rmax = 96, 64, 12, 0.08
    say("nn distances in a graph")
    src_np = _random_set(4000, W, H, T, 11)
    qry_np = _random_set(3000, W, H, T, 12)
    src, qry = Q.to_device(src_np), Q.to_device(qry_np)
    scratch = torch.empty(int(B.load().esim_nn_scratch_bytes(W, H, T)), dtype=torch.uint8, device="cuda")
    B.nn_distances(src, qry, W, H, T, rmax, scratch=scratch)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.nn_distances(src, qry, W, H, T, rmax, scratch=scratch)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = B.nn_distances(src, qry, W, H, T, rmax, scratch=scratch)
    rng = np.random.default_rng(5)
    for k in range(3):
        if k:
            # move the source events: a stale bitmap would keep the old ones
            src["x"].copy_(torch.from_numpy(rng.integers(0, W, src_np["x"].size).astype(np.int32)).cuda())
        g.replay()
        torch.cuda.synchronize()
        ref = B.nn_distances(src, qry, W, H, T, rmax, scratch=torch.empty_like(scratch))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
        _ = (ref * 2).sum().item()
