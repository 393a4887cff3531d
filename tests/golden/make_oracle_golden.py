"""Writes oracle_small_workload.json: the oracle's results on the small seeded
workload (64x64x16, F = 7, r = 5, tr = 0, C = 0.2), as a regression record of
the oracle itself.

These values are not pins: they come from the oracle, and the oracle is pinned
by the closed forms, invariants, library routines and brute force of the
test_oracle_*.py files.  The record makes any later change of the oracle's
arithmetic visible (the stored digests stop matching), so that such a change
has to be made on purpose.  Only the oracle and the seeded input generator are
called.

    python tests/golden/make_oracle_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2303_02608_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small_workload.json")
# (t, px, py) of the stored regressions: corners, an edge, the centre, a late frame
REGRESSIONS = [(0, 0, 0), (0, 63, 0), (0, 5, 60), (0, 31, 32), (7, 40, 20), (15, 63, 63)]
MODES = {"thresholded": oracle.THRESHOLDED, "exhaustive": oracle.EXHAUSTIVE, "raw": oracle.RAW}


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def record() -> dict:
    cfg = synth.config_spec(0)
    d = synth.make_clip(cfg["spec"])
    E, feat = d["E"].numpy(), d["feat"].numpy()
    y = oracle.log_brightness(E)
    oc = oracle.Clip(y, feat)
    p = oracle.Params(cfg["r"], cfg["tr"], cfg["C"])
    out = {"workload": "small: 64x64x16, 4 spp, F = 7 f32, r = 5, tr = 0, C = 0.2 (seeded synthetic clip)",
           "inputs": {"E_sha256": sha(E.astype(np.float32)), "feat_sha256": sha(feat.astype(np.float32)),
                      "y_sha256": sha(np.asarray(y, np.float64))}}
    for name, mode in MODES.items():
        o = oracle.run(oc, p, mode, want_dl=True)
        x, yy, t, pol = o["events"]
        ev = np.stack([np.asarray(t, np.int64), np.asarray(yy, np.int64), np.asarray(x, np.int64),
                       np.asarray(pol, np.int64)], axis=1)
        out[name] = {"count": int(o["count"]), "events_sha256": sha(ev), "dl_sha256": sha(np.asarray(o["dl"], np.float64)),
                     "first": ev[:5].tolist(), "last": ev[-5:].tolist()}
    regs = []
    for t, px, py in REGRESSIONS:
        theta, info = oracle.regress(oc, p, t, px, py)
        regs.append({"t": t, "px": px, "py": py, "theta": [repr(float(v)) for v in theta],
                     "W": repr(float(info["W"])), "R": repr(float(info["R"]))})
    out["regressions"] = regs
    return out


if __name__ == "__main__":
    rec = record()
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}")
