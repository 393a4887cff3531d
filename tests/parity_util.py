"""Helpers shared by the GPU parity tests: running the HIP path through the
C ABI and comparing its events with the oracle's.

Event parity rule: per pixel, the GPU's event frames and polarities must equal
the oracle's until the first frame where they differ; that frame is excused
only if the oracle's compared change |dL| lies within `band` of C (rounding
can then legitimately flip the decision), after which the pixel's states
diverge and it is excused for the rest of the clip.  Any other difference is a
failure."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd.simulator import Simulator

MODE_ID = {"thresholded": oracle.THRESHOLDED, "exhaustive": oracle.EXHAUSTIVE, "raw": oracle.RAW}


def say(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(E: np.ndarray, feat: np.ndarray):
    Ed = torch.from_numpy(np.ascontiguousarray(E, dtype=np.float32)).cuda()
    fd = torch.from_numpy(np.ascontiguousarray(feat)).cuda()
    y = B.log_brightness(Ed)
    return y, fd


def oracle_clip(E: np.ndarray, feat: np.ndarray):
    return oracle.Clip(oracle.log_brightness(E), feat)


def compare_events(gpu: dict, orc: dict, W: int, C: float, band: float = 1e-4,
                   pixels=None):
    """Returns (n_compared_pixels, n_excused, failures[list]).  Vectorised:
    pixels whose (frame, polarity) histories agree exactly are settled with
    array operations; only the others are examined one by one."""
    ox, oy, ot, op = orc["events"]
    dl = orc["dl"]                      # [T][npix] in the oracle's pixel order
    pix_list = np.asarray(orc["pixels"] if orc.get("pixels") is not None else np.arange(dl.shape[1]))
    check = np.asarray(pix_list if pixels is None else pixels, dtype=np.int64)

    def ordered(x, y, t, p):
        pix = np.asarray(y, np.int64) * W + np.asarray(x, np.int64)
        keep = np.isin(pix, check)
        pix, t, p = pix[keep], np.asarray(t, np.int64)[keep], np.asarray(p, np.int64)[keep]
        o = np.lexsort((t, pix))
        return pix[o], t[o], p[o]

    gpix, gt, gp = ordered(gpu["x"], gpu["y"], gpu["t"], gpu["p"])
    opix, ot_, op_ = ordered(ox, oy, ot, op)
    npx = int(check.max(initial=0)) + 1
    cg = np.bincount(gpix, minlength=npx)
    co = np.bincount(opix, minlength=npx)
    bad = cg != co
    same = ~bad
    mg, mo = same[gpix], same[opix]
    mism = (gt[mg] != ot_[mo]) | (gp[mg] != op_[mo])
    bad[gpix[mg][mism]] = True
    fails, excused = [], 0
    for q in check[bad[check]]:
        q = int(q)
        gi = {int(t): int(pp) for t, pp in zip(gt[gpix == q], gp[gpix == q])}
        oi = {int(t): int(pp) for t, pp in zip(ot_[opix == q], op_[opix == q])}
        first = min(t for t in set(gi) | set(oi) if gi.get(t) != oi.get(t))
        d = dl[first, int(np.searchsorted(pix_list, q))]
        if np.isfinite(d) and abs(abs(d) - C) <= band:
            excused += 1
        else:
            fails.append((q, first, gi.get(first), oi.get(first), float(d)))
    return int(check.size), excused, fails


def run_gpu(E, feat, params: B.Params, mode: str, capacity=None, keep_dl=False):
    y, fd = to_dev(E, feat)
    sim = Simulator(y, fd, params, capacity=capacity)
    if not keep_dl:
        return sim.run(mode), sim
    # frame loop by hand so the per-frame dl can be kept
    T, HW = sim.T, sim.HW
    dls = np.full((T, HW), np.nan)
    p, n = sim.plan, HW
    sim.ev.count.zero_()
    if mode == "thresholded":
        B.regress(p, 0, None, None, n, sim.alpha, sim.beta)
        B.events(p, 0, B.INIT, None, alpha=sim.alpha, beta=sim.beta, n_out=n)
        for t in range(1, T):
            B.threshold(p, t, sim.dl, sim.worklist, sim.count)
            B.regress(p, t, sim.worklist, sim.count, n, sim.alpha, sim.beta)
            B.events(p, t, B.THRESHOLDED, sim.ev, worklist=sim.worklist, count=sim.count,
                     dl=sim.dl, alpha=sim.alpha, beta=sim.beta, n_out=n)
            dls[t] = sim.dl.cpu().numpy()
    elif mode == "exhaustive":
        for t in range(T):
            B.regress(p, t, None, None, n, sim.alpha, None)
            B.events(p, t, B.EXHAUSTIVE, sim.ev, dl=sim.dl, alpha=sim.alpha, n_out=n)
            if t:
                dls[t] = sim.dl.cpu().numpy()
    else:
        for t in range(T):
            B.events(p, t, B.RAW, sim.ev, dl=sim.dl)
            if t:
                dls[t] = sim.dl.cpu().numpy()
    torch.cuda.synchronize()
    out = sim.events()
    out["dl"] = dls
    return out, sim


def compare_every_crossing(gpu: dict, orc: dict, L: np.ndarray, W: int, C: float, dt: float = 1.0,
                           band: float = 1e-4, pixels=None, ts_abs: float = 1e-5,
                           ts_rel: float = 5e-5):
    """Every-crossing events (several per pixel-frame, interpolated times) of
    the GPU against the oracle's (modes RAW_ALL / EXHAUSTIVE_ALL).

    Per pixel, the (frame, polarity) sequences must be equal up to the first
    frame where they differ; that frame is excused only if the oracle's
    compared change |d| lies within `band` of a level k C (k >= 1), after which
    the pixel is excused.  Before it, every event time must agree within
    ts_abs * max(1, t) + ts_rel / |L_t - L_{t-1}| frames (the FP32 rounding of
    the time, plus the brightness error over the frame's slope), scaled by dt.
    L: [T][npix] the oracle's compared values (y, or its alpha) in the oracle's
    pixel order.  Returns (n_compared, n_excused, failures, max time error)."""
    ox, oy, ot, op = orc["events"]
    dl = orc["dl"]
    pix_list = np.asarray(orc["pixels"] if orc.get("pixels") is not None else np.arange(dl.shape[1]))
    check = np.asarray(pix_list if pixels is None else pixels, dtype=np.int64)

    def ordered(x, y, t, p, ts):
        pix = y.astype(np.int64) * W + x
        keep = np.isin(pix, check)
        pix, t, p, ts = pix[keep], t[keep].astype(np.int64), p[keep].astype(np.int64), ts[keep]
        o = np.lexsort((t, pix))          # stable: the crossings of a pixel-frame keep their order
        return pix[o], t[o], p[o], ts[o]

    gpix, gt, gp, gts = ordered(gpu["x"], gpu["y"], gpu["t"], gpu["p"], np.asarray(gpu["ts"], np.float64))
    opix, ot_, op_, ots = ordered(ox, oy, ot, op, np.asarray(orc["ts"], np.float64) * dt)
    npx = int(max(check.max(initial=0), 0)) + 1
    cg = np.bincount(gpix, minlength=npx)
    co = np.bincount(opix, minlength=npx)
    same_n = cg == co
    mg = same_n[gpix]
    mo = same_n[opix]
    # pixels with equal counts: events align one to one in the sorted order
    bad = np.zeros(npx, bool)
    mism = (gt[mg] != ot_[mo]) | (gp[mg] != op_[mo])
    bad[gpix[mg][mism]] = True
    bad |= ~same_n
    # times of the pixels whose sequences agree completely
    good_ev = ~bad[opix]
    col = np.searchsorted(pix_list, opix[good_ev])
    te = ot_[good_ev]
    slope = np.abs(L[te, col] - L[te - 1, col])
    err = np.abs(gts[~bad[gpix]] - ots[good_ev])
    tol = dt * (ts_abs * np.maximum(1, te) + ts_rel / np.maximum(slope, 1e-30))
    fails, excused = [], 0
    max_err = float(err.max() / dt) if err.size else 0.0
    for i in np.nonzero(err > tol)[0][:10]:
        fails.append((int(opix[good_ev][i]), int(te[i]), "time", float(gts[~bad[gpix]][i]),
                      float(ots[good_ev][i])))
    # pixels whose sequences differ: the first differing frame must be in the band
    for pix in np.nonzero(bad[check])[0]:
        q = int(check[pix])
        a = np.nonzero(gpix == q)[0]
        b = np.nonzero(opix == q)[0]
        n = 0
        while n < a.size and n < b.size and gt[a[n]] == ot_[b[n]] and gp[a[n]] == op_[b[n]]:
            n += 1
        cand = ([gt[a[n]]] if n < a.size else []) + ([ot_[b[n]]] if n < b.size else [])
        first = int(min(cand))
        c = int(np.searchsorted(pix_list, q))
        for i in range(n):
            t = int(ot_[b[i]])
            if t >= first:
                break
            e = abs(gts[a[i]] - ots[b[i]])
            max_err = max(max_err, e / dt)
            if e > dt * (ts_abs * max(1, t) + ts_rel / max(abs(L[t, c] - L[t - 1, c]), 1e-30)):
                fails.append((q, t, "time", float(gts[a[i]]), float(ots[b[i]])))
                break
        d = abs(dl[first, c])
        k = max(1.0, np.round(d / C))
        if np.isfinite(d) and abs(d - k * C) <= band:
            excused += 1
        else:
            fails.append((q, first, "events", float(d)))
    return int(check.size), excused, fails, max_err
