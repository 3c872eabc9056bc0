import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def hz():
    """The HIP library's Python binding on cuda:0 (fails loudly if not built)."""
    if not gpu_available():
        pytest.fail("a GPU test ran without a visible HIP device")
    import paper_1712_08743_amd as hzpkg
    return hzpkg
