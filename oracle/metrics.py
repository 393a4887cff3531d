"""Event-set comparison of Sec. 3 ("Quantitative comparison"), plain and slow.

Test infrastructure only: imported by tests/, the smoke check and the bench's
quality workload, never by the product path.

Each event set is a set of signed points (x, y, t) with polarity p.  Points
are compared in the scaled coordinates (x sx, y sy, t st); the reading taken
here is sx = 1/W, sy = 1/H, st = 1/T (every axis normalised to [0, 1]), since
the paper does not state the units of its distance threshold.

  d(e -> S)   distance from e to the closest event of S with the same polarity
              (+inf when there is none within rmax)
  P(tau)      share of generated events g with d(g -> R) < tau   (eq. precision)
  R(tau)      share of reference events r with d(r -> G) < tau   (eq. recall)
  F(tau)      harmonic mean of P and R
  CD          mean of d(g -> R)^2 over G plus mean of d(r -> G)^2 over R: the
              point-set Chamfer distance of RPM-Net made polarity-aware as the
              paper describes; a distance beyond rmax counts as rmax (a reading:
              the paper does not say how unmatched points enter)

The nearest neighbour is a library primitive (scipy's cKDTree), per polarity.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def scaled(x, y, t, W, H, T):
    return np.stack([np.asarray(x, np.float64) / W, np.asarray(y, np.float64) / H,
                     np.asarray(t, np.float64) / T], axis=1)


def nn_distances(src, qry, W, H, T, rmax):
    """src, qry: dicts of x, y, t, p arrays.  For every query event the distance
    to the nearest source event of the same polarity, +inf beyond rmax."""
    n = len(qry["x"])
    out = np.full(n, np.inf)
    for pol in (1, -1):
        sm = np.asarray(src["p"]) == pol
        qm = np.asarray(qry["p"]) == pol
        if not sm.any() or not qm.any():
            continue
        tree = cKDTree(scaled(np.asarray(src["x"])[sm], np.asarray(src["y"])[sm],
                              np.asarray(src["t"])[sm], W, H, T))
        d, _ = tree.query(scaled(np.asarray(qry["x"])[qm], np.asarray(qry["y"])[qm],
                                 np.asarray(qry["t"])[qm], W, H, T), k=1)
        d = np.where(d <= rmax, d, np.inf)
        out[np.nonzero(qm)[0]] = d
    return out


def metrics(gen, ref, W, H, T, taus, rmax):
    """P, R, F at every tau and the polarity-aware Chamfer distance."""
    dg = nn_distances(ref, gen, W, H, T, rmax)     # generated -> reference
    dr = nn_distances(gen, ref, W, H, T, rmax)     # reference -> generated
    out = {"P": [], "R": [], "F": []}
    for tau in taus:
        P = float(np.mean(dg < tau)) if dg.size else 0.0
        R = float(np.mean(dr < tau)) if dr.size else 0.0
        out["P"].append(P)
        out["R"].append(R)
        out["F"].append(2 * P * R / (P + R) if P + R > 0 else 0.0)
    cg = np.minimum(dg, rmax) ** 2
    cr = np.minimum(dr, rmax) ** 2
    out["CD"] = float((cg.mean() if cg.size else 0.0) + (cr.mean() if cr.size else 0.0))
    return out
