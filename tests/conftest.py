import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(autouse=True)
def _canaries(request):
    """GPU tests: every hog.Buffers a test (or bench.py under it) makes gets
    guard bands, checked after the test (hog_cases.GuardedBuffers)."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    from paper_1703_06256_amd import hog
    import hog_cases
    orig = hog.Buffers
    hog.Buffers = hog_cases.GuardedBuffers
    try:
        yield
    finally:
        hog.Buffers = orig
    hog_cases.check_all_guards()
