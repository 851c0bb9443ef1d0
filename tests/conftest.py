import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (ROCm device) and the built librbe.so")
    config.addinivalue_line("markers", "slow: long CPU statistical test")


@pytest.fixture(scope="session")
def gpu():
    """Fail loudly (not skip) when a GPU test runs without a device or library."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no ROCm device is visible")
    from paper_2110_14362_amd import rbe
    rbe.load_library()
    return torch.device("cuda:0")
