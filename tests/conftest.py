import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle check")


def pytest_collection_modifyitems(session, config, items):
    config._hfqmc_gpu_selected = any(it.get_closest_marker("gpu") for it in items)


@pytest.fixture(scope="session", autouse=True)
def _torch_runtime_first(request):
    # PyTorch ships its own HIP runtime; it must initialise the device before the
    # library's runtime does, or it finds no GPU.  Only when GPU tests run.
    if getattr(request.config, "_hfqmc_gpu_selected", False):
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    yield
