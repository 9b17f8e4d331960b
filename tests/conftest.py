import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gfq_gpu():
    """The bound HIP library on cuda:0; fails loudly (never falls back) if it is missing."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    from paper_0901_1413_amd import gfq
    gfq.load()
    return gfq
