import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.Oracle.lib()  # builds only if the library is missing or stale
    return oracle
