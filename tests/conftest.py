import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")


def make_cluster(pos, species, box=60.0, pbc=(0, 0, 0)):
    """One structure from explicit positions (a large cubic cell)."""
    from workloads import make_batch
    pos = np.asarray(pos, dtype=np.float32)
    return make_batch([(pos, np.asarray(species, dtype=np.int32), np.eye(3) * box, pbc)])


@pytest.fixture
def cluster():
    return make_cluster
