import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: statistical oracle pins that take tens of seconds")


@pytest.fixture(autouse=True)
def _single_threaded_blas(request):
    """CPU tests run numpy's BLAS on one thread.  The oracle's matrices are
    small (a few hundred rows at most), and a BLAS thread pool per product
    costs more in start-up and spinning than the product itself: the
    3000-seed unbiasedness pin took 277 s with the pool and 28 s without."""
    if request.node.get_closest_marker("gpu") is not None:
        yield
        return
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"):
        yield
