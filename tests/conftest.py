import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (large oracle solves)")
    # the oracle's host worker server starts before any test touches the GPU
    from oracle import pool
    pool.start()


@pytest.fixture(scope="session")
def gpu_lib():
    """The loaded HIP library; the GPU tests fail loudly if it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_1208_5435_amd import mfipm
    return mfipm.load_library()
