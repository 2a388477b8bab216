import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(autouse=True)
def _oracle_blas_one_thread(request):
    """GPU tests run the oracle beside the device: its many small least-squares
    solves are fastest, and do not contend with the host threads that drive
    the device, on one BLAS thread."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        yield
