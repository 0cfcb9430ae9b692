import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def ssp():
    """The ctypes binding of the HIP library (built in-tree first if it is missing)."""
    from paper_2511_03343_amd import ssp as binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2511_03343_amd import build
        build.build()
    binding.lib()
    return binding


@pytest.fixture(scope="session")
def gpu(ssp):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.init()
    return torch
