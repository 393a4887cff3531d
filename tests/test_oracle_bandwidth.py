"""Pins of the bandwidth-optimised regression in the oracle (Sec. 3, bandwidth
optimisation: the global bandwidth h of eq. 5 chosen per regression by an
estimate of alpha's mean squared error from the MC variance).

  - SURE is unbiased: averaged over many noise realisations of a known smooth
    scene, SURE_k equals the mean of (alpha_k - f_c)^2 within Monte Carlo error,
    for every candidate h.
  - The hat weight in SURE is d alpha / d y_c: recovered from two SURE values
    it equals the finite difference of alpha under a change of y_c.
  - Noise-free affine data (ridge 0): every candidate fits exactly, SURE = 0
    up to rounding and theta is the affine map.
  - The delta-method variance of log(mean) against simulated sample means.
"""
import numpy as np
import pytest

import oracle
from paper_2303_02608_amd import synth


def _scene(W=7, H=7, T=1, F=2, seed=5):
    d = synth.random_features_clip(W, H, T, F, seed)
    feat = d["feat"].numpy()
    rng = np.random.default_rng(seed)
    g = rng.uniform(-1, 1, size=F)
    # smooth but not affine in the features: a curvature term makes the bias
    # grow with h while the variance falls
    f = (0.3 + np.einsum("f,tfhw->thw", g, feat.astype(np.float64))
         + 1.5 * feat[:, 0].astype(np.float64) ** 2)
    return f, feat


def test_sure_is_unbiased_for_every_candidate():
    f, feat = _scene()
    T, F, H, W = feat.shape
    hs = np.array([0.3, 0.6, 1.2])
    sigma2 = np.full((T, H, W), 0.04)
    c = (0 * H + 3) * W + 3
    fc = f[0, 3, 3]
    p = oracle.Params(r=2, tr=0, C=1.0)
    rng = np.random.default_rng(17)
    N = 1500
    sure = np.empty((N, hs.size))
    err2 = np.empty((N, hs.size))
    for k in range(N):
        y = f + np.sqrt(sigma2) * rng.standard_normal(f.shape)
        out = oracle.regress_bandwidth(oracle.Clip(y, feat), p, hs, sigma2, np.array([c]), nthreads=1)
        sure[k] = out["sure"][0]
        err2[k] = (out["alpha_k"][0] - fc) ** 2
    d = sure - err2
    se = d.std(axis=0, ddof=1) / np.sqrt(N)
    assert np.all(np.abs(d.mean(axis=0)) <= 4 * se), (d.mean(axis=0), se)
    # the candidates' risks differ, so the choice matters
    risk = err2.mean(axis=0)
    assert risk.max() > 1.5 * risk.min()


def test_hat_weight_is_the_derivative_of_alpha():
    f, feat = _scene(seed=8)
    T, F, H, W = feat.shape
    hs = np.array([0.5, 1.0, 2.0])
    c, py, px = 2 * W + 4, 2, 4
    p = oracle.Params(r=2, tr=0, C=1.0, ridge=1e-3)
    s = 0.01
    zero = np.zeros((T, H, W))
    var = np.full((T, H, W), s)
    a = oracle.regress_bandwidth(oracle.Clip(f, feat), p, hs, zero, np.array([c]))
    b = oracle.regress_bandwidth(oracle.Clip(f, feat), p, hs, var, np.array([c]))
    ell = (b["sure"][0] - a["sure"][0] + s) / (2 * s)
    delta = 1e-3
    f2 = f.copy()
    f2[0, py, px] += delta
    a2 = oracle.regress_bandwidth(oracle.Clip(f2, feat), p, hs, zero, np.array([c]))
    fd = (a2["alpha_k"][0] - a["alpha_k"][0]) / delta
    assert np.allclose(ell, fd, rtol=1e-6, atol=1e-9)
    assert np.all((ell > 0) & (ell <= 1.0))
    # and it falls as the bandwidth widens (more neighbours share the weight)
    assert ell[0] > ell[1] > ell[2]


def test_affine_data_every_candidate_exact():
    T, F, H, W = 1, 3, 8, 8
    d = synth.random_features_clip(W, H, T, F, 9)
    feat = d["feat"].numpy()
    rng = np.random.default_rng(9)
    g = rng.uniform(-2, 2, size=F)
    y = 0.4 + np.einsum("f,tfhw->thw", g, feat.astype(np.float64))
    hs = np.array([0.4, 1.0, 2.5])
    p = oracle.Params(r=2, tr=0, C=1.0, ridge=0.0)
    items = np.arange(H * W)
    out = oracle.regress_bandwidth(oracle.Clip(y, feat), p, hs, np.zeros((T, H, W)), items)
    # SURE is zero up to rounding for every candidate (which one wins is
    # decided by rounding), and whichever wins carries the exact fit
    assert np.max(np.abs(out["sure"])) <= 1e-20
    assert np.allclose(out["alpha_k"], y.reshape(-1)[:, None], atol=1e-12)
    th = out["theta"]
    assert np.allclose(th[:, 0], y.reshape(-1), atol=1e-12)
    assert np.allclose(th[:, 3:], g[None, :], atol=1e-9)
    assert np.allclose(th[:, 1:3], 0.0, atol=1e-9)


def test_choice_is_the_smallest_sure():
    f, feat = _scene(W=9, H=8, seed=21)
    T, F, H, W = feat.shape
    rng = np.random.default_rng(3)
    y = f + 0.1 * rng.standard_normal(f.shape)
    hs = np.array([0.35, 0.7, 1.4, 2.8])
    vy = np.full(f.shape, 0.01)
    out = oracle.regress_bandwidth(oracle.Clip(y, feat), oracle.Params(r=3, tr=0, C=1.0), hs, vy,
                                   np.arange(H * W))
    k = np.argmin(out["sure"], axis=1)
    assert np.array_equal(out["h"], hs[k])
    assert np.allclose(out["theta"][:, 0], out["alpha_k"][np.arange(H * W), k])
    assert len(set(k.tolist())) > 1


def test_log_variance_delta_method():
    E = np.array([1.0, 0.25, 3.0], np.float32)
    var = np.array([1.0, 0.0625, 9.0], np.float32)
    vy = oracle.log_variance(E, var, 64)
    assert np.allclose(vy, var / 64 / (E.astype(np.float64) + 1e-3) ** 2, rtol=1e-15)
    # against simulated means of 64 unit exponentials: Var[log mean] ~ 1/64
    rng = np.random.default_rng(0)
    m = rng.exponential(1.0, size=(20000, 64)).mean(axis=1)
    assert np.log(m).var() == pytest.approx(vy[0], rel=0.06)
