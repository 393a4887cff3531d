"""Batched conversion of clips of uneven size, length and radius in one plan:
bitwise equal to converting each clip alone, and matching the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from paper_2303_02608_amd.simulator import BatchSimulator, Simulator
from parity_util import compare_events, oracle_clip, say, to_dev

pytestmark = pytest.mark.gpu


def _clips():
    # radii up to 9: a work list with 16 lanes per item then mixes the one-pass
    # instance (windows of at most 16 columns) with the general one
    shapes = [(40, 30, 9, 3, 1), (64, 48, 6, 2, 1), (23, 57, 12, 4, 0), (50, 50, 3, 3, 1),
              (64, 64, 10, 5, 1), (36, 28, 5, 9, 1)]
    out = []
    for i, (W, H, T, r, tr) in enumerate(shapes):
        spec = synth.ClipSpec(W=W, H=H, T=T, spp=2 + i, F=7, n_discs=2 + i, speed=(0.5, 2.0),
                              seed=5000 + i)
        d = synth.make_clip(spec)
        out.append((d["E"].numpy(), d["feat"].numpy(), B.Params(r=r, tr=tr, C=0.2)))
    return out


def _key(x, y, t, p):
    return list(zip(t.tolist(), y.tolist(), x.tolist(), p.tolist()))


def test_batch_equals_single_clips_and_oracle():
    clips = _clips()
    say(f"batch of {len(clips)} clips")
    devs = [to_dev(E, f) for E, f, _ in clips]
    bs = BatchSimulator([y for y, _ in devs], [f for _, f in devs], [p for *_, p in clips])
    for sched in [(4, 16, 1), (4, 4, 2), (2, 8, 4)]:
        bs.plan.set_schedule(*sched)
        got = bs.run()
        assert got["count"] > 0
        # one esim_step per frame == separate threshold / regress / events calls
        sep = bs.run(fused=False)
        for k in ("x", "y", "t", "p", "clip"):
            assert np.array_equal(got[k], sep[k]), (sched, k)
        for c, ((E, feat, p), (y, fd)) in enumerate(zip(clips, devs)):
            m = got["clip"] == c
            single = Simulator(y, fd, p).run("thresholded")
            assert _key(got["x"][m], got["y"][m], got["t"][m], got["p"][m]) == \
                _key(single["x"], single["y"], single["t"], single["p"]), (sched, c)
        # order: (t, clip, py, px)
        k = (got["t"].astype(np.int64) << 40) + (got["clip"].astype(np.int64) << 28) + \
            got["y"].astype(np.int64) * 4096 + got["x"]
        assert np.all(np.diff(k) > 0)
    for c, (E, feat, p) in enumerate(clips):
        m = got["clip"] == c
        orc = oracle.run(oracle_clip(E, feat), oracle.Params(p.r, p.tr, p.C), oracle.THRESHOLDED,
                         want_dl=True)
        g = {k: got[k][m] for k in ("x", "y", "t", "p")}
        n, exc, fails = compare_events(g, orc, feat.shape[3], p.C, 1e-4)
        assert not fails and exc <= 2, (c, fails[:5])


def test_batch_graph_replay():
    # radii 3, 2 and 9: the step's work list is split in two segments
    clips = [_clips()[k] for k in (0, 1, 5)]
    say("batch graph replay")
    devs = [to_dev(E, f) for E, f, _ in clips]
    bs = BatchSimulator([y for y, _ in devs], [f for _, f in devs], [p for *_, p in clips])
    eager = bs.run()
    bs.capture()
    for _ in range(3):
        bs.graph.replay()
        torch.cuda.synchronize()
        got = bs.ev.host()
        for k in ("x", "y", "t", "p", "clip"):
            assert np.array_equal(got[k], eager[k])


@pytest.mark.parametrize("radii", [(5, 8), (8, 5, 6)])
def test_split_work_list_with_chunked_prefix(radii):
    """Plans of more than 4096 flag blocks (the prefix goes through chunk
    totals) with windows on both sides of 16 columns: the step's two list
    segments give the events of each clip converted alone, bit for bit, in
    (t, clip, py, px) order."""
    say(f"split work list, chunked prefix, radii {radii}")
    ys, fs, ps = [], [], []
    for i, r in enumerate(radii):
        spec = synth.ClipSpec(W=1024, H=600, T=4, spp=2, F=7, n_discs=12, speed=(1.0, 3.0),
                              seed=5100 + i)
        d = synth.make_clip(spec, device="cuda")
        ys.append(B.log_brightness(d["E"]))
        fs.append(d["feat"])
        ps.append(B.Params(r=r, tr=1, C=0.2))
    bs = BatchSimulator(ys, fs, ps)
    assert bs.plan.npix // 256 > 4096
    got = bs.run()
    assert got["count"] > 0
    sep = bs.run(fused=False)
    for k in ("x", "y", "t", "p", "clip"):
        assert np.array_equal(got[k], sep[k]), k
    for c, (y, f, p) in enumerate(zip(ys, fs, ps)):
        m = got["clip"] == c
        single = Simulator(y, f, p).run("thresholded")
        assert m.sum() > 0
        assert _key(got["x"][m], got["y"][m], got["t"][m], got["p"][m]) == \
            _key(single["x"], single["y"], single["t"], single["p"]), c
    k = (got["t"].astype(np.int64) << 40) + (got["clip"].astype(np.int64) << 28) + \
        got["y"].astype(np.int64) * 4096 + got["x"]
    assert np.all(np.diff(k) > 0)
