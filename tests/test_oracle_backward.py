"""Pins of the oracle's adjoint of alpha (eqs. 4-5 differentiated) against
central finite differences of the oracle's forward regression and against
closed-form invariants of weighted least squares."""
import numpy as np
import pytest

import oracle
from paper_2303_02608_amd import synth


def _clip(W=10, H=9, T=3, F=3, seed=7):
    d = synth.random_features_clip(W, H, T, F, seed)
    return oracle.Clip(oracle.log_brightness(d["E"].numpy()), d["feat"].numpy())


def _loss(clip, p, items, ga):
    out = oracle.regress_items(clip, p, items)
    return float(np.dot(ga, out["theta"][:, 0]))


@pytest.mark.parametrize("ridge,b", [(1e-6, None), (1e-2, [1.0, 1.3, 0.7, 1.1, 0.9])])
def test_adjoint_matches_central_differences(ridge, b):
    clip = _clip()
    p = oracle.Params(r=2, tr=1, C=0.2, h=1.0, b=b, ridge=ridge)
    HW = clip.H * clip.W
    rng = np.random.default_rng(3)
    items = np.unique(rng.integers(0, clip.T * HW, size=12))
    ga = rng.standard_normal(items.size)
    gy, gb, fails = oracle.backward(clip, p, items, ga)
    assert fails == 0
    hstep = 1e-3
    # y entries: pick some inside the windows of the items and some outside
    flat = clip.y.reshape(-1)
    cand = np.concatenate([np.nonzero(gy.reshape(-1))[0][:10], [0, flat.size - 1]])
    for q in cand:
        old = flat[q]
        flat[q] = old + hstep
        lp = _loss(clip, p, items, ga)
        flat[q] = old - hstep
        lm = _loss(clip, p, items, ga)
        flat[q] = old
        fd = (lp - lm) / (2 * hstep)
        assert gy.reshape(-1)[q] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    bb = np.ones(clip.D) if b is None else np.array(b, float)
    for j in range(clip.D):
        bp = bb.copy()
        bp[j] += hstep
        lp = _loss(clip, oracle.Params(p.r, p.tr, p.C, p.h, bp, p.ridge), items, ga)
        bm = bb.copy()
        bm[j] -= hstep
        lm = _loss(clip, oracle.Params(p.r, p.tr, p.C, p.h, bm, p.ridge), items, ga)
        fd = (lp - lm) / (2 * hstep)
        assert gb[j] == pytest.approx(fd, rel=2e-5, abs=1e-8)


def test_alpha_weights_sum_to_one_and_are_orthogonal_to_u():
    """The hat-matrix row of alpha reproduces constants (sum_i d alpha/d y_i = 1,
    any beta-only ridge) and, with lambda = 0, linear functions of x
    (sum_i (d alpha/d y_i) u_ij = 0)."""
    clip = _clip(F=2, seed=9)
    HW = clip.H * clip.W
    for ridge in (0.0, 1e-3):
        p = oracle.Params(r=2, tr=1, C=0.2, ridge=ridge)
        for (t, px, py) in [(1, 4, 4), (0, 0, 0), (2, 9, 8)]:
            item = np.array([t * HW + py * clip.W + px])
            gy, gb, _ = oracle.backward(clip, p, item, np.ones(1))
            assert gy.sum() == pytest.approx(1.0, abs=1e-12)
            if ridge == 0.0:
                pos, w, z = oracle.window(clip, p, t, px, py)
                coef = gy[pos[:, 0], pos[:, 1], pos[:, 2]]
                np.testing.assert_allclose(coef @ z[:, 1:], 0.0, atol=1e-11)


def test_bandwidth_gradient_vanishes_on_affine_data():
    """With y affine in x and lambda = 0 the fit is exact for every weighting,
    so alpha does not depend on b."""
    F, r = 3, 2
    d = synth.random_features_clip(9, 8, 2, F, seed=13)
    feat = d["feat"].numpy()
    g = np.array([0.4, -0.2, 1.2, -0.8, 0.5])
    py, px = np.meshgrid(np.arange(8), np.arange(9), indexing="ij")
    y = 0.1 + g[0] * px / r + g[1] * py / r + np.einsum("f,tfhw->thw", g[2:], feat.astype(np.float64))
    clip = oracle.Clip(y, feat)
    p = oracle.Params(r=r, tr=1, C=0.2, ridge=0.0)
    items = np.array([0, 17, 40, 72 + 33])
    gy, gb, fails = oracle.backward(clip, p, items, np.ones(items.size))
    assert fails == 0
    np.testing.assert_allclose(gb, 0.0, atol=1e-10)
