import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU run")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    if not oracle.LIB.exists():
        oracle.build()
    oracle.set_threads(min(8, os.cpu_count() or 1))
    return oracle
