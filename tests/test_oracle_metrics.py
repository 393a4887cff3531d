"""Pins of the event-set comparison (Sec. 3, quantitative comparison) in the
oracle: cases whose precision, recall, F1 and Chamfer distance follow from the
definitions by hand, and brute force on small random sets."""
import numpy as np
import pytest

from oracle import metrics as M

W, H, T = 40, 30, 20
RMAX = 0.2


def _random_set(n, seed):
    rng = np.random.default_rng(seed)
    return dict(x=rng.integers(0, W, n), y=rng.integers(0, H, n), t=rng.integers(0, T, n),
                p=rng.choice([-1, 1], n))


def test_identical_sets():
    g = _random_set(300, 1)
    m = M.metrics(g, g, W, H, T, [1e-6, 0.01], RMAX)
    assert m["P"] == [1.0, 1.0] and m["R"] == [1.0, 1.0] and m["F"] == [1.0, 1.0]
    assert m["CD"] == 0.0


def test_one_pixel_shift():
    g = _random_set(200, 2)
    g["x"] = np.clip(g["x"], 0, W - 2)
    r = dict(g, x=g["x"] + 1)
    d = M.nn_distances(r, g, W, H, T, RMAX)
    # the shifted copy of each event is at distance 1/W; another reference event
    # of the same polarity may be closer only if it sits at the same point
    assert np.all(d <= 1.0 / W + 1e-15)
    m = M.metrics(g, r, W, H, T, [0.5 / W, 1.5 / W], RMAX)
    assert m["P"][1] == 1.0 and m["R"][1] == 1.0


def test_single_pair_by_hand():
    # (0,0,0) and (3,4,0) on a 10x10x10 lattice: distance sqrt(0.3^2 + 0.4^2) = 0.5
    g = dict(x=np.array([0]), y=np.array([0]), t=np.array([0]), p=np.array([1]))
    r = dict(x=np.array([3]), y=np.array([4]), t=np.array([0]), p=np.array([1]))
    d = M.nn_distances(r, g, 10, 10, 10, 1.0)
    assert d[0] == pytest.approx(0.5, abs=1e-15)
    m = M.metrics(g, r, 10, 10, 10, [0.49, 0.51], 1.0)
    assert m["P"] == [0.0, 1.0] and m["R"] == [0.0, 1.0] and m["F"] == [0.0, 1.0]
    assert m["CD"] == pytest.approx(0.5, abs=1e-14)        # 0.25 + 0.25
    # beyond rmax the distance is infinite and the Chamfer term is capped at rmax^2
    m = M.metrics(g, r, 10, 10, 10, [0.6], 0.4)
    assert m["P"] == [0.0] and m["CD"] == pytest.approx(2 * 0.16, abs=1e-14)


def test_polarity_is_respected():
    g = _random_set(100, 3)
    r = dict(g, p=-g["p"])
    d = M.nn_distances(r, g, W, H, T, 0.5 / W)
    # every same-position event has the other polarity: nothing within half a pixel
    assert np.all(np.isinf(d))


def test_against_brute_force():
    g = _random_set(150, 4)
    r = _random_set(170, 5)
    d = M.nn_distances(r, g, W, H, T, RMAX)
    for i in range(len(g["x"])):
        same = r["p"] == g["p"][i]
        dd = np.sqrt((((r["x"][same] - g["x"][i]) / W) ** 2 + ((r["y"][same] - g["y"][i]) / H) ** 2 +
                      ((r["t"][same] - g["t"][i]) / T) ** 2))
        best = dd.min() if dd.size else np.inf
        best = best if best <= RMAX else np.inf
        assert d[i] == pytest.approx(best, abs=1e-14) or (np.isinf(d[i]) and np.isinf(best))
