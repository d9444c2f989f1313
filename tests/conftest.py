import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def torch_gpu_runtime_first(request):
    """GPU sessions initialise torch's HIP runtime before the first call into
    libpm, as bench.py does.  The process then holds two HIP runtimes
    (torch's and the one libpm links); with libpm's initialised first, a
    later first use of torch's failed to find the GPU after some sequences of
    tests (the anisotropic file, then the gradient workload)."""
    gpu = any(item.get_closest_marker("gpu") for item in request.session.items)
    if gpu:
        try:
            import torch
        except ImportError:
            torch = None
        if torch is not None and torch.cuda.is_available():
            torch.cuda.init()
            torch.empty(1, device="cuda")
    yield
