"""Frame loop of the event simulator on the GPU.

Three conversions of a clip (y = log brightness [T][H][W], feat [T][F][H][W]):

* ``"thresholded"`` -- the paper's method (Sec. 2.2): regress every pixel at
  frame 0, then per frame threshold (Prop. 1), regress only the flagged pixels
  and emit their events.
* ``"exhaustive"`` -- WLR+ESIM (Sec. 3): regress every pixel of every frame,
  then eq. (1) on the regressed values.
* ``"raw"`` -- ESIM on the noisy frames (Sec. 3): eq. (1) on y.

Every step is a libesim call enqueued on one stream; the loop never
synchronises, so it can be captured in a hipGraph and replayed.  By default a
frame is one esim_step call (threshold, compaction with the events, and the
list regression writing the state: three launches); ``fused=False`` runs the
same frame through the separate threshold / regress / events calls, which also
leave the work list and the regression outputs in this object's buffers.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding as B

MODES = ("thresholded", "exhaustive", "raw")


class Simulator:
    def __init__(self, y: torch.Tensor, feat: torch.Tensor, params: B.Params,
                 capacity: Optional[int] = None, want_dl: bool = True, with_ts: Optional[bool] = None):
        T, F, H, W = feat.shape
        self.T, self.F, self.H, self.W = T, F, H, W
        self.HW = H * W
        dev = feat.device
        self.plan = B.Plan([y], [feat], [params])
        self.state = self.plan.states[0]
        self.dl = torch.empty(self.HW, dtype=torch.float32, device=dev)
        self.worklist = torch.empty(self.plan.wl_capacity, dtype=torch.int64, device=dev)
        self.count = torch.zeros(2, dtype=torch.int32, device=dev)
        self.alpha = torch.empty(self.HW, dtype=torch.float32, device=dev)
        self.beta = torch.empty((F + 2, self.HW), dtype=torch.float32, device=dev)
        if capacity is None:
            capacity = min(T * self.HW, 1 << 26)
        # event times t * dt (every-crossing events: their interpolated times);
        # kept by default only for the every-crossing rule
        self.ev = B.Events(capacity, dev, with_ts=params.multi_crossing if with_ts is None else with_ts)
        # per-frame flagged counts (only recorded when asked: it adds a copy per frame)
        self.flagged = torch.zeros(T, dtype=torch.int32, device=dev)
        self.graph = None
        self.graph_mode = None

    # -- one conversion, enqueued on the current stream --------------------
    def enqueue(self, mode: str = "thresholded", record_flags: bool = False, fused: bool = True):
        if mode not in MODES:
            raise ValueError(mode)
        p, n = self.plan, self.HW
        self.ev.count.zero_()
        if fused and not record_flags:
            if mode == "thresholded":
                B.step(p, 0, B.INIT)
                for t in range(1, self.T):
                    B.step(p, t, B.THRESHOLDED, self.ev, self.dl)
            else:
                m = B.EXHAUSTIVE if mode == "exhaustive" else B.RAW
                for t in range(self.T):
                    B.step(p, t, m, self.ev, self.dl)
            return
        if mode == "thresholded":
            B.regress(p, 0, None, None, n, self.alpha, self.beta)
            B.events(p, 0, B.INIT, None, alpha=self.alpha, beta=self.beta, n_out=n)
            for t in range(1, self.T):
                B.threshold(p, t, self.dl, self.worklist, self.count)
                if record_flags:
                    self.flagged[t:t + 1].copy_(self.count[1:2])
                B.regress(p, t, self.worklist, self.count, n, self.alpha, self.beta)
                B.events(p, t, B.THRESHOLDED, self.ev, worklist=self.worklist, count=self.count,
                         dl=self.dl, alpha=self.alpha, beta=self.beta, n_out=n)
        elif mode == "exhaustive":
            for t in range(self.T):
                B.regress(p, t, None, None, n, self.alpha, None)
                B.events(p, t, B.EXHAUSTIVE, self.ev, dl=self.dl, alpha=self.alpha, n_out=n)
        else:
            for t in range(self.T):
                B.events(p, t, B.RAW, self.ev, dl=self.dl)

    def capture(self, mode: str = "thresholded", fused: bool = True):
        """Record one conversion into a hipGraph (torch.cuda.CUDAGraph)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue(mode, fused=fused)          # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.enqueue(mode, fused=fused)
        self.graph, self.graph_mode = g, mode
        return g

    def replay(self):
        self.graph.replay()

    def run(self, mode: str = "thresholded", fused: bool = True):
        self.enqueue(mode, fused=fused)
        torch.cuda.synchronize()
        return self.events()

    def events(self):
        return self.ev.host()


class BatchSimulator:
    """The thresholded conversion of many clips of uneven size and length in
    one plan: every step launches one threshold, one work-list regression and
    one event call over all clips still running (a clip of length T takes part
    in steps 0..T-1).  Events carry their clip index."""

    def __init__(self, ys, feats, params, capacity: Optional[int] = None):
        self.plan = B.Plan(list(ys), list(feats), list(params))
        dev = feats[0].device
        self.T = max(int(f.shape[0]) for f in feats)
        self.npix = self.plan.npix
        self.n_out = max(self.plan.npix, self.plan.wl_capacity)
        self.dl = torch.empty(self.npix, dtype=torch.float32, device=dev)
        self.worklist = torch.empty(self.plan.wl_capacity, dtype=torch.int64, device=dev)
        self.count = torch.zeros(2, dtype=torch.int32, device=dev)
        self.alpha = torch.empty(self.n_out, dtype=torch.float32, device=dev)
        self.beta = torch.empty((self.plan.D, self.n_out), dtype=torch.float32, device=dev)
        if capacity is None:
            capacity = min(sum(int(f.shape[0]) * f.shape[2] * f.shape[3] for f in feats), 1 << 27)
        self.ev = B.Events(capacity, dev, with_clip=True)

    def enqueue(self, fused: bool = True):
        p, n = self.plan, self.n_out
        self.ev.count.zero_()
        if fused:
            B.step(p, 0, B.INIT)
            for t in range(1, self.T):
                B.step(p, t, B.THRESHOLDED, self.ev, self.dl)
            return
        B.regress(p, 0, None, None, n, self.alpha, self.beta)
        B.events(p, 0, B.INIT, None, alpha=self.alpha, beta=self.beta, n_out=n)
        for t in range(1, self.T):
            B.threshold(p, t, self.dl, self.worklist, self.count)
            B.regress(p, t, self.worklist, self.count, n, self.alpha, self.beta)
            B.events(p, t, B.THRESHOLDED, self.ev, worklist=self.worklist, count=self.count,
                     dl=self.dl, alpha=self.alpha, beta=self.beta, n_out=n)

    def capture(self, fused: bool = True):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue(fused)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.enqueue(fused)
        self.graph = g
        return g

    def run(self, fused: bool = True):
        self.enqueue(fused)
        torch.cuda.synchronize()
        return self.ev.host()
