"""Boundary checks that need a plan (and so a device): size guards of the
per-item-frame calls, the output length of thresholded events, and the event
times t * dt."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd.simulator import Simulator
from parity_util import say, to_dev

pytestmark = pytest.mark.gpu


def _dummy_plan(W, H, T, F, f16):
    """A plan over a clip whose arrays are never read: every call below is
    rejected by validation before anything is enqueued."""
    lib = B.load()
    clip = B.esim_clip(W, H, T, F, B.F16 if f16 else B.F32, 256, 256)
    par = B.Params(r=3, tr=1, C=0.2).struct(F)
    st = B.State(H, W, F, "cuda")
    sts = st.struct()
    h = ctypes.c_void_p()
    assert lib.esim_plan_create(ctypes.byref(clip), ctypes.byref(par), ctypes.byref(sts), 1,
                                ctypes.byref(h)) == B.OK, lib.esim_last_error()
    return lib, h, st


def test_brightness_over_4gib_is_rejected_for_per_item_frames():
    # F = 1 in FP16: the features (2 B per pixel-frame) stay below 4 GiB while
    # the brightness (4 B per pixel-frame) does not
    W, H, T = 1024, 1024, 1025
    assert T * W * H * 2 < 1 << 32 <= T * W * H * 4
    say("4 GiB brightness guard")
    lib, h, st = _dummy_plan(W, H, T, 1, True)
    try:
        a = torch.empty(4, device="cuda")
        wl = torch.zeros(4, dtype=torch.int64, device="cuda")
        cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
        rc = lib.esim_wlr_regress(h, -1, wl.data_ptr(), cnt.data_ptr(), 4, a.data_ptr(), None, None, None, None)
        assert rc == B.E_UNSUPPORTED, lib.esim_last_error()
        gb = torch.zeros(3, dtype=torch.float64, device="cuda")
        rc = lib.esim_wlr_backward(h, wl.data_ptr(), 4, a.data_ptr(), a.data_ptr(), gb.data_ptr(),
                                   a.data_ptr(), 1 << 40, None)
        assert rc == B.E_UNSUPPORTED, lib.esim_last_error()
        # a uniform frame only reads the 2 tr + 1 frames of its window: allowed
        assert lib.esim_backward_scratch_bytes(h, 4) > 0
    finally:
        lib.esim_plan_destroy(h)


def test_thresholded_events_need_outputs_for_every_listed_item(small_clip):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    say("thresholded events n_out check")
    y, fd = to_dev(E, feat)
    sim = Simulator(y, fd, B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"]))
    HW = sim.HW
    B.regress(sim.plan, 0, None, None, HW, sim.alpha, sim.beta)
    B.events(sim.plan, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=HW)
    B.threshold(sim.plan, 1, sim.dl, sim.worklist, sim.count)
    with pytest.raises(B.EsimError) as e:
        B.events(sim.plan, 1, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count, dl=sim.dl,
                 alpha=sim.alpha, beta=sim.beta, n_out=HW - 1)
    assert e.value.status == B.E_INVAL
    # nothing was enqueued: the event count is untouched
    torch.cuda.synchronize()
    assert int(sim.ev.count.item()) == 0


@pytest.mark.parametrize("multi", [False, True])
def test_event_times_are_frame_times_dt(small_clip, multi):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    dt = 1e-3
    say(f"event times t * dt, multi_crossing={multi}")
    y, fd = to_dev(E, feat)
    T = feat.shape[0]
    outs = []
    for d in (1.0, dt):
        sim = Simulator(y, fd, B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"], dt=d, multi_crossing=multi),
                        capacity=8 * T * sim_hw(feat), with_ts=True)
        outs.append(sim.run("raw"))
    a, b = outs
    assert a["count"] == b["count"] > 0
    for k in ("x", "y", "t", "p"):
        assert np.array_equal(a[k], b[k])
    assert np.allclose(b["ts"], (a["ts"].astype(np.float64) * dt).astype(np.float32), rtol=1e-6, atol=0)
    if not multi:
        assert np.array_equal(b["ts"], (b["t"].astype(np.float64) * dt).astype(np.float32))


def sim_hw(feat):
    return feat.shape[2] * feat.shape[3]
