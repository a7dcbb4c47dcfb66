import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def rfd():
    """The HIP library binding; GPU tests fail loudly if it cannot load."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    import paper_2601_18835_amd as pkg
    return pkg
