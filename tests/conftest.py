import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    # long CPU pins (paper-table rows of the largest chaos sizes) run with SGPC_RUN_SLOW=1
    if os.environ.get("SGPC_RUN_SLOW") != "1":
        slow = pytest.mark.skip(reason="long CPU pin: set SGPC_RUN_SLOW=1 to run")
        for item in items:
            if "slow" in item.keywords:
                item.add_marker(slow)
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(autouse=True)
def _release_gpu_handles(request):
    """After each GPU test: release the library handles the test dropped (their
    finalisers run now, while the runtime is up, not at interpreter exit) and
    wait for the device."""
    yield
    if "gpu" not in request.keywords or not _gpu_available():
        return
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
