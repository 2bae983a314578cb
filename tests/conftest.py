import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# under pytest-xdist, share the cores between the workers instead of letting
# every worker's torch start one thread per core
if os.environ.get("PYTEST_XDIST_WORKER"):
    import torch
    _workers = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1"))
    torch.set_num_threads(max(1, (os.cpu_count() or 1) // max(1, _workers)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its Python binding; GPU tests fail loudly
    (rather than skip) if the GPU is visible but the library is missing."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    from paper_2312_07725_amd import nsfr
    return nsfr
