"""The reduced-precision regression (ESIM_GRAM_F32C: FP32 regressors and
Gram with block-compensated sums, FP64 re-solve above the condition bound)
and FP16 feature storage, with their errors stated per output against the
FP64 oracle.  Parity for this variant is unpinned beyond these stated bounds:
it is an accuracy/speed option, not the contract path."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from parity_util import oracle_clip, say, to_dev

pytestmark = pytest.mark.gpu


def _run(E, feat, p, t, lanes=4):
    y, fd = to_dev(E, feat)
    plan = B.Plan([y], [fd], [p])
    plan.set_schedule(lanes, lanes, 4)
    HW = plan.npix
    a = torch.empty(HW, device="cuda")
    b = torch.empty((plan.D, HW), device="cuda")
    R = torch.empty(HW, device="cuda")
    K = torch.empty(HW, device="cuda")
    B.regress(plan, t, None, None, HW, a, b, R, K)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), R.cpu().numpy(), K.cpu().numpy()


def _errors(out, E, feat, p, t):
    clip = oracle_clip(E, feat)
    HW = clip.H * clip.W
    ref = oracle.regress_items(clip, oracle.Params(p.r, p.tr, p.C, p.h, p.b, p.ridge), t * HW + np.arange(HW))
    th = ref["theta"]
    a, b, R, K = out
    ea = np.abs(a - th[:, 0]) / np.maximum(1, np.abs(th[:, 0]))
    eb = np.abs(b.T - th[:, 1:]) / np.maximum(1, np.abs(th[:, 1:]))
    er = np.abs(R - ref["R"])
    return ea, eb, er


@pytest.mark.parametrize("lanes", [4, 16])
def test_compensated_fp32_errors_small_workload(small_clip, lanes):
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    for bound in (1e6, 1e3):
        p = B.Params(r=cfg["r"], tr=1, C=cfg["C"], precision=B.GRAM_F32C, kappa_fp64=bound)
        say(f"f32c lanes={lanes} bound={bound:g}")
        out = _run(E, feat, p, 5, lanes)
        ea, eb, er = _errors(out, E, feat, p, 5)
        frac = np.mean(out[3] > bound)
        say(f"f32c bound {bound:g}: fp64 re-solves {frac:.3%}; alpha err max {ea.max():.2e} "
            f"p99 {np.quantile(ea, 0.99):.2e}; beta err max {eb.max():.2e}; R err max {er.max():.2e}")
        assert np.all(np.isfinite(out[0]))
        # stated bounds for this workload (FP32 Gram; the contract path is FP64)
        assert ea.max() <= 2e-3
        assert np.quantile(ea, 0.99) <= 2e-4


def test_f16_feature_storage_errors(small_clip):
    """FP16 storage: the FP64 path on FP16-rounded features matches the oracle
    on the same FP16 values (arithmetic error), and the storage error against
    the FP32 features is stated."""
    E, feat32, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    feat16 = feat32.astype(np.float16)
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    say("f16 storage")
    out = _run(E, feat16, p, 4)
    ea, eb, er = _errors(out, E, feat16, p, 4)
    assert ea.max() <= 1e-4 and eb.max() <= 1e-4
    es, _, _ = _errors(out, E, feat32, p, 4)
    say(f"f16 storage: arithmetic alpha err {ea.max():.2e}; storage alpha err max {es.max():.2e} "
        f"p99 {np.quantile(es, 0.99):.2e}")
    assert np.quantile(es, 0.5) <= 1e-2
