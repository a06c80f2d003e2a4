import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def geo():
    from paper_1712_09407_amd import synth
    return (synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)


def event_dict(e):
    return dict(y=e.y, z=e.z, row_offsets=e.row_offsets, sector_id=e.sector_id)


def f32(v):
    """The FP32 value of a parameter, widened: both trackers see the same number."""
    return float(np.float32(v))
