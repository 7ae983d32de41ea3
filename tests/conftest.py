import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP GPU (MI355X) and the built libtd.so")
    config.addinivalue_line("markers", "slow: long-running")


@pytest.fixture(scope="session")
def td():
    """The HIP binding, loaded; skips nothing: a GPU test fails loudly if the
    library or the device is missing."""
    import torch
    import paper_1409_3901_amd as td
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    td.load()
    return td


@pytest.fixture(scope="session")
def dev():
    import torch
    return torch.device("cuda:0")


# Options of the three kernels the parity tests cover: the plain float64
# tier, the float32-filtered tier with the bucketed sweep (the default) and
# the filtered tier with the full bitonic sort.
PREC_OPTS = {
    "plain": dict(precision="plain"),
    "filtered": dict(precision="filtered"),
    "bitonic": dict(precision="filtered", sweep="bitonic"),
}


def to_dev(a, dev):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
