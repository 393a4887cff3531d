"""The oracle against its own stored results on the small workload
(tests/golden/oracle_small_workload.json, written by make_oracle_golden.py in
the same folder): a regression record, not a pin.  A mismatch means the
oracle's arithmetic (or the input generator, checked first) changed."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_oracle_golden as G  # noqa: E402


@pytest.fixture(scope="module")
def stored():
    with open(G.OUT) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def now():
    return G.record()


def test_inputs_unchanged(stored, now):
    assert now["inputs"] == stored["inputs"]


@pytest.mark.parametrize("mode", ["thresholded", "exhaustive", "raw"])
def test_events_and_dl_unchanged(stored, now, mode):
    assert now["inputs"] == stored["inputs"], "the input generator changed"
    assert now[mode] == stored[mode]


def test_regressions_unchanged(stored, now):
    assert now["regressions"] == stored["regressions"]
