"""Every-crossing events (ESIM with interpolated times, the multi_crossing
option of the exhaustive and raw modes) against the oracle's rule, on the same
FP32 compared values (y for raw, the GPU's per-frame alpha for exhaustive):
positions, frames and polarities exactly, times to FP32 rounding."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd.simulator import Simulator
from parity_util import say, to_dev

pytestmark = pytest.mark.gpu


def _check(gpu, orc):
    assert gpu["count"] == orc["count"] > 0
    assert len(gpu["x"]) == gpu["count"]
    for k in ("x", "y", "t", "p"):
        assert np.array_equal(gpu[k], orc[k]), k
    assert np.max(np.abs(gpu["ts"] - orc["ts"])) <= 2e-6
    # times lie in (t - 1, t] and increase within a pixel-frame
    assert np.all((gpu["ts"] > gpu["t"] - 1) & (gpu["ts"] <= gpu["t"] + 1e-6))


@pytest.mark.parametrize("C", [0.05, 0.2])
def test_raw_multicrossing_matches_oracle(small_clip, C):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=C, multi_crossing=True)
    say(f"raw every-crossing C={C}")
    y, fd = to_dev(E, feat)
    T, F, H, W = feat.shape
    orc = oracle.esim_multi_crossing(y.cpu().numpy().reshape(T, H * W), C, W)
    # several events per pixel-frame: size the sink from the oracle's count
    sim = Simulator(y, fd, p, capacity=orc["count"] + 1024)
    gpu = sim.run("raw")
    say(f"events {gpu['count']} (one-per-frame rule would allow at most {(T - 1) * H * W})")
    _check(gpu, orc)
    # the state: L_ref quantised to the crossed levels, last = the final frame
    assert torch.equal(sim.state.last, y[T - 1].reshape(-1))


def test_exhaustive_multicrossing_matches_oracle(small_clip):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    C = 0.1
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=C, multi_crossing=True)
    say("exhaustive every-crossing")
    y, fd = to_dev(E, feat)
    T, F, H, W = feat.shape
    HW = H * W
    sim = Simulator(y, fd, p, capacity=8 * T * HW)
    alphas = np.empty((T, HW), np.float32)
    sim.ev.count.zero_()
    for t in range(T):
        B.regress(sim.plan, t, None, None, HW, sim.alpha, None)
        alphas[t] = sim.alpha.cpu().numpy()
        B.events(sim.plan, t, B.EXHAUSTIVE, sim.ev, dl=sim.dl, alpha=sim.alpha, n_out=HW)
    torch.cuda.synchronize()
    _check(sim.events(), oracle.esim_multi_crossing(alphas, C, W))


@pytest.mark.parametrize("mode", ["raw", "exhaustive"])
def test_multicrossing_step_and_graph(small_clip, mode):
    """The step entry point equals the separate calls bit for bit, and graph
    replays reproduce the eager run."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=0.1, multi_crossing=True)
    say(f"every-crossing step vs separate calls, {mode}")
    y, fd = to_dev(E, feat)
    T, F, H, W = feat.shape
    a = Simulator(y, fd, p, capacity=8 * T * H * W)
    b = Simulator(y, fd, p, capacity=8 * T * H * W)
    ea = a.run(mode, fused=True)
    assert ea["count"] <= a.ev.capacity
    eb = b.run(mode, fused=False)
    for k in ("x", "y", "t", "p", "ts"):
        assert np.array_equal(ea[k], eb[k]), k
    assert torch.equal(a.state.alpha, b.state.alpha) and torch.equal(a.state.last, b.state.last)
    a.capture(mode)
    for _ in range(2):
        a.replay()
        torch.cuda.synchronize()
        g = a.events()
        for k in ("x", "y", "t", "p", "ts"):
            assert np.array_equal(g[k], ea[k]), k
        _ = (y * 2).sum().item()
