import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    stale = (not os.path.exists(oracle.LIB_PATH) or
             os.path.getmtime(oracle.LIB_PATH) < os.path.getmtime(oracle.SRC_PATH))
    if stale:
        oracle.build()
    return oracle
