import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.environ.get("GS_ORACLE_LIB"):
        oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def c0():
    import gsgen
    return gsgen.config0()


@pytest.fixture(scope="session")
def c1():
    import gsgen
    return gsgen.config1()


@pytest.fixture(scope="session")
def c2():
    import gsgen
    return gsgen.config2()
