"""Event-set comparison of Sec. 3 ("Quantitative comparison") on the GPU.

Events are signed points (x, y, t) compared in coordinates normalised by
(W, H, T).  With d(e -> S) the distance from e to the closest event of S with
the same polarity (esim_nn_distances, exact within rmax):

  P(tau) = share of generated events with d(g -> R) < tau
  R(tau) = share of reference events with d(r -> G) < tau
  F(tau) = 2 P R / (P + R)
  CD     = mean d(g -> R)^2 + mean d(r -> G)^2 (RPM-Net's Chamfer distance made
           polarity-aware), distances beyond rmax counted as rmax.

The nearest-neighbour search is the library's kernel; the shares and means are
reductions over its output.
"""
from __future__ import annotations

from typing import Dict, Iterable

import numpy as np
import torch

from . import binding as B


def to_device(ev: Dict[str, np.ndarray], device="cuda") -> Dict[str, torch.Tensor]:
    return {"x": torch.as_tensor(np.asarray(ev["x"], np.int32), device=device),
            "y": torch.as_tensor(np.asarray(ev["y"], np.int32), device=device),
            "t": torch.as_tensor(np.asarray(ev["t"], np.int32), device=device),
            "p": torch.as_tensor(np.asarray(ev["p"], np.int8), device=device)}


def metrics(gen: Dict[str, torch.Tensor], ref: Dict[str, torch.Tensor], W: int, H: int, T: int,
            taus: Iterable[float], rmax: float, keep: bool = False) -> Dict[str, object]:
    """P, R, F per tau and CD; with ``keep`` also the per-event distances
    ``dg`` (generated -> reference) and ``dr`` (reference -> generated)."""
    dg = B.nn_distances(ref, gen, W, H, T, rmax)     # generated -> reference
    dr = B.nn_distances(gen, ref, W, H, T, rmax)     # reference -> generated
    out = {"P": [], "R": [], "F": []}
    for tau in taus:
        P = float((dg < tau).double().mean()) if dg.numel() else 0.0
        R = float((dr < tau).double().mean()) if dr.numel() else 0.0
        out["P"].append(P)
        out["R"].append(R)
        out["F"].append(2 * P * R / (P + R) if P + R > 0 else 0.0)
    cg = torch.clamp(dg, max=rmax) ** 2
    cr = torch.clamp(dr, max=rmax) ** 2
    out["CD"] = float((cg.mean() if cg.numel() else 0.0) + (cr.mean() if cr.numel() else 0.0))
    if keep:
        out["dg"], out["dr"] = dg, dr
    return out
