"""Schedule autotuner of the regression kernel.

The regression kernel has two schedule knobs per plan (esim_plan_set_schedule):
the number of lanes that share one regression item (dense launches and
work-list launches separately) and the persistent blocks per CU.  More lanes
per item means more, shorter wave tasks, which pays off for the sparse per-frame
work lists of the thresholded path; dense launches prefer fewer lanes (no
cross-lane reduction, no idle column lanes, the solve shared by 64 items).

The tuner replays a short prefix of the real conversion (frame 0 dense, then a
few thresholded frames) once per candidate and times only the regression
launches with HIP events on the launch stream.  Results are cached per clip
shape and parameters for the life of the process.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import binding as B

_cache: Dict[tuple, Tuple[int, int, int]] = {}


def _key(plan: B.Plan, frames: int):
    parts = []
    for y, f, p in zip(plan.ys, plan.feats, plan.params):
        parts.append((tuple(f.shape), str(f.dtype), p.r, p.tr, p.C, p.precision))
    return (tuple(parts), frames)


def _time_prefix(plan: B.Plan, frames: int, bufs) -> Tuple[float, float]:
    """Runs frame 0 (dense) and frames 1..frames-1 (thresholded) of every clip
    of the plan; returns (dense regress ms, summed work-list regress ms)."""
    dl, wl, cnt, a, b, ev = bufs
    n_out = a.numel()
    stream = torch.cuda.current_stream()
    ev.count.zero_()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    B.regress(plan, 0, None, None, n_out, a, b)
    e1.record(stream)
    B.events(plan, 0, B.INIT, None, alpha=a, beta=b, n_out=n_out)
    marks = []
    for t in range(1, frames):
        B.threshold(plan, t, dl, wl, cnt)
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        B.regress(plan, t, wl, cnt, n_out, a, b)
        s1.record(stream)
        marks.append((s0, s1))
        B.events(plan, t, B.THRESHOLDED, ev, worklist=wl, count=cnt, dl=dl, alpha=a, beta=b,
                 n_out=n_out)
    torch.cuda.synchronize()
    dense = e0.elapsed_time(e1)
    # the first frames flag few pixels; weigh the later ones
    lst = sum(x.elapsed_time(y) for x, y in marks[len(marks) // 2:])
    return dense, lst


def tune(plan: B.Plan, frames: int = 12, lanes_dense: Iterable[int] = (1, 2, 4),
         lanes_list: Iterable[int] = (4, 8, 16), blocks_per_cu: Iterable[int] = (1, 2, 4, 8),
         reps: int = 2, verbose: bool = False) -> Tuple[int, int, int]:
    """Pick (lanes_dense, lanes_list, blocks_per_cu) for the plan and apply it.

    The plan's states are overwritten (the prefix is a real conversion)."""
    key = _key(plan, frames)
    if key in _cache:
        plan.set_schedule(*_cache[key])
        return _cache[key]
    dev = plan.feats[0].device
    n_out = max(plan.npix, plan.wl_capacity)
    bufs = (torch.empty(plan.npix, dtype=torch.float32, device=dev),
            torch.empty(plan.wl_capacity, dtype=torch.int64, device=dev),
            torch.zeros(2, dtype=torch.int32, device=dev),
            torch.empty(n_out, dtype=torch.float32, device=dev),
            torch.empty((plan.D, n_out), dtype=torch.float32, device=dev),
            B.Events(1 << 16, dev))
    frames = max(2, min(frames, min(f.shape[0] for f in plan.feats)))
    best_dense: Dict[int, float] = {}
    best_list: Dict[Tuple[int, int], float] = {}
    for ld, ll, bpc in itertools.product(lanes_dense, lanes_list, blocks_per_cu):
        if ld != 1 and ll != 16:
            continue          # tuned along the lines through (1, 16) only
        try:
            plan.set_schedule(ld, ll, bpc)
        except B.EsimError:
            continue          # no kernel instance for this combination
        _time_prefix(plan, frames, bufs)            # warm-up
        d = l = float("inf")
        for _ in range(reps):
            dd, llm = _time_prefix(plan, frames, bufs)
            d, l = min(d, dd), min(l, llm)
        best_dense[(ld, bpc)] = min(best_dense.get((ld, bpc), float("inf")), d)
        best_list[(ll, bpc)] = min(best_list.get((ll, bpc), float("inf")), l)
        if verbose:
            print(f"[autotune] dense L={ld} list L={ll} bpc={bpc}: dense {d:.3f} ms, list {l:.3f} ms",
                  flush=True)
    # one blocks_per_cu for both launch kinds: minimise the weighted total
    T = min(f.shape[0] for f in plan.feats)
    nlist = max(1, (frames - 1) - (frames - 1) // 2)
    best = None
    for bpc in blocks_per_cu:
        if not any(b_ == bpc for (_, b_) in best_dense):
            continue
        dl_ = min((v, L) for (L, b_), v in best_dense.items() if b_ == bpc)
        ll_ = min((v, L) for (L, b_), v in best_list.items() if b_ == bpc)
        total = dl_[0] + ll_[0] / nlist * (T - 1)
        if best is None or total < best[0]:
            best = (total, dl_[1], ll_[1], bpc)
    sched = (best[1], best[2], best[3])
    plan.set_schedule(*sched)
    _cache[key] = sched
    return sched
