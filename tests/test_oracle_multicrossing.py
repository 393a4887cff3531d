"""Pins of the every-crossing event rule (ESIM proper) in the oracle: a
brightness ramp fires at closed-form levels and times; a monotone sequence
fires floor(|L_T - L_0| / C) events in all; reversals flip the polarity; below
C nothing fires."""
import numpy as np
import pytest

import oracle


def test_ramp_closed_form():
    C, s, L0 = 0.25, 0.6, -1.0          # 2.4 C per frame
    T = 6
    L = (L0 + s * np.arange(T, dtype=np.float64))[:, None].astype(np.float32)
    ev = oracle.esim_multi_crossing(L, C, 1)
    Lf = L[:, 0].astype(np.float64)
    # levels L0 + k C crossed at t = (L0 + k C - L0) / s
    kmax = int(np.floor((Lf[-1] - Lf[0]) / C + 1e-12))
    assert ev["count"] == kmax
    k = np.arange(1, kmax + 1)
    t_cross = (k * C) / s
    assert np.all(ev["p"] == 1)
    assert np.allclose(ev["ts"], t_cross, atol=2e-6)
    # the frame of each event is the first frame at or after its crossing
    assert np.array_equal(ev["t"], np.ceil(t_cross - 1e-9).astype(np.int32))


def test_monotone_total_and_order():
    rng = np.random.default_rng(0)
    T, n = 30, 50
    L = np.cumsum(rng.uniform(0.0, 0.9, (T, n)), axis=0).astype(np.float32)
    C = 0.3
    ev = oracle.esim_multi_crossing(L, C, n)
    for q in range(n):
        m = ev["x"] == q
        # telescoping: the reference moves by whole steps of C
        assert m.sum() == int(np.floor((np.float64(L[-1, q]) - np.float64(L[0, q])) / C))
        assert np.all(np.diff(ev["ts"][m]) > 0)
        assert np.all((ev["ts"][m] > ev["t"][m] - 1) & (ev["ts"][m] <= ev["t"][m] + 1e-6))


def test_reversal_and_below_threshold():
    C = 0.5
    L = np.array([[0.0], [1.2], [1.4], [0.1], [0.2]], np.float32)
    ev = oracle.esim_multi_crossing(L, C, 1)
    # 0 -> 1.2: crossings at 0.5, 1.0 (ref 1.0); 1.4: none; 0.1: d = -0.9 -> one at 0.5 (ref 0.5);
    # 0.2: d = -0.3 -> none
    assert list(ev["t"]) == [1, 1, 3]
    assert list(ev["p"]) == [1, 1, -1]
    assert ev["ts"][0] == pytest.approx(0.5 / 1.2, abs=1e-6)
    assert ev["ts"][1] == pytest.approx(1.0 / 1.2, abs=1e-6)
    assert ev["ts"][2] == pytest.approx(2 + (1.4 - 0.5) / 1.3, abs=1e-6)
