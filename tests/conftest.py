import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: PU200-sized CPU work (tens of seconds)")


@pytest.fixture(scope="session")
def barrel():
    from lstgen import barrel_geometry
    return barrel_geometry()


@pytest.fixture(scope="session")
def full():
    from lstgen import full_geometry
    return full_geometry()


@pytest.fixture(scope="session")
def obarrel(barrel):
    import oracle
    return oracle.OracleGeometry(barrel)


@pytest.fixture(scope="session")
def ofull(full):
    import oracle
    return oracle.OracleGeometry(full)
