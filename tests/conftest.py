import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

if hasattr(sys, "set_int_max_str_digits"):
    sys.set_int_max_str_digits(0)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its C ABI (skips when no GPU is present)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_09301_amd import mpts
    return mpts
