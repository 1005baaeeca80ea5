import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True)
def _release_cached_device_memory(request):
    """After each GPU test, return the caching allocator's free blocks to the
    device: the large tests need workspaces of over 100 GiB in one piece."""
    yield
    if request.node.get_closest_marker("gpu") is None or "torch" not in sys.modules:
        return
    torch = sys.modules["torch"]
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        import gc

        gc.collect()
        torch.cuda.empty_cache()
