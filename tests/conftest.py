import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


@pytest.fixture(scope="session")
def gpu_lib():
    """The device library through its C-ABI binding; fails loudly when the GPU or the build is missing."""
    import paper_1704_05528_amd as svt
    svt.require_gpu()
    return svt
