import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def sky_map():
    """The synthetic 2048x1024 sky with a 0.5 deg sun (generated once per session)."""
    from paper_2305_20061_amd import synth
    return synth.env_map()


@pytest.fixture(scope="session")
def small_sky():
    """A 256x128 sky with the same generator (sun enlarged by resolution)."""
    from paper_2305_20061_amd import synth
    return synth.env_map(256, 128)


def rel_rmse(g, o):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return float(np.sqrt(np.sum((g - o) ** 2)) / np.sqrt(np.sum(o ** 2)))
