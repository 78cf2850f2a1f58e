import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def pytest_runtest_logstart(nodeid, location):
    # name the case before it runs, so a run that dies on the GPU still says which
    if "gpu" in nodeid:
        sys.__stderr__.write(f"[start] {nodeid}\n")
        sys.__stderr__.flush()


@pytest.fixture(scope="session")
def orc():
    """The C oracle, built once per session if it is not built yet."""
    import oracle
    if not os.path.exists(oracle.oracle.LIB):
        oracle.build()
    return oracle
