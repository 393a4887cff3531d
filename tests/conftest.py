import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running")


@pytest.fixture(scope="session")
def small_clip():
    """The small workload (64x64x16, 4 spp, F=7, r=5, Tr=0, C=0.2) as numpy."""
    from paper_2303_02608_amd import synth
    cfg = synth.config_spec(0)
    d = synth.make_clip(cfg["spec"])
    return dict(E=d["E"].numpy(), feat=d["feat"].numpy(), cfg=cfg)
