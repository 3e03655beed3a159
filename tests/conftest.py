import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libnsc.so")
    config.addinivalue_line("markers", "slow: longer oracle runs")


@pytest.fixture(autouse=True)
def _release_device_memory(request):
    """After each GPU test: drop its contexts and hand torch's cached blocks
    back to the device, so that the full-size workloads of later tests (up
    to ~230 GiB each) find the memory free."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    import gc

    import torch
    gc.collect()
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
