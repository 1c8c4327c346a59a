import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(autouse=True)
def _no_setup_retries(request):
    """GPU tests: no mesh freed during the test needed a repeated setup factorisation (the
    library retries a failed element-block or coarse Cholesky once and counts it)."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    try:
        import paper_1907_01572_amd as hp
    except ImportError:
        yield
        return
    start = len(hp.RETRY_LOG)
    yield
    retried = [r for r in hp.RETRY_LOG[start:] if r != (0, 0)]
    assert not retried, "setup factorisations were repeated: %s" % retried
