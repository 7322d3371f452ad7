import os
import sys

import pytest

# torch first: libhb then binds to the HIP runtime that torch ships, so torch's device
# tensors and streams are valid in the library's calls within one test process
try:
    import torch  # noqa: F401
except ImportError:
    pass

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workloads (minutes of oracle time)")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def hb():
    """The GPU binding; fails loudly when the HIP library is missing."""
    import paper_1504_02687_amd as pkg
    pkg.load()
    return pkg
