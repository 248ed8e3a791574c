import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); runs the HIP path")
    config.addinivalue_line("markers", "slow: long-running case")


def pytest_report_header(config):
    return "paper_2012_05695_amd tests (root %s)" % ROOT


@pytest.fixture(scope="session")
def libddm_path():
    """Path of the built library; builds it in-tree if it is missing (CPU-only build)."""
    from paper_2012_05695_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    return b.LIB


@pytest.fixture(scope="session")
def gpu():
    """Skips nothing: a GPU test that finds no device must fail, not pass silently."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible HIP device"
    from paper_2012_05695_amd import api  # raises if libddm.so is missing
    return api
