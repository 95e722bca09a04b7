import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test (oracle at larger sizes)")


def has_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; GPU tests only."""
    if not has_gpu():
        pytest.skip("no GPU")
    import paper_1704_00865_amd as wf
    wf.load()  # raises if the extension is missing
    return wf
