import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The CPU oracle runs OpenMP loops.  Idle OpenMP threads should sleep, not
# spin (several test processes may share the cores), and pytest-xdist workers
# split the cores between them.  Set before the oracle library is loaded.
os.environ.setdefault("OMP_WAIT_POLICY", "passive")
if "PYTEST_XDIST_WORKER_COUNT" in os.environ:
    _workers = max(1, int(os.environ["PYTEST_XDIST_WORKER_COUNT"]))
    os.environ.setdefault("OMP_NUM_THREADS", str(max(1, (os.cpu_count() or 1) // _workers)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle
