import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for path in (ROOT, os.path.join(ROOT, "tests")):
    if path not in sys.path:
        sys.path.insert(0, path)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: runs HIP kernels on an MI355X (gfx950) device")


@pytest.fixture(scope="session")
def device():
    """The HIP device; GPU tests fail (not skip) when there is none."""
    import torch

    assert torch.cuda.is_available(), "GPU test run without a HIP device"
    return torch.device("cuda:0")
