import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# the planted-mistake test points this at a modified copy of the oracle package
if os.environ.get("ORACLE_PY_DIR"):
    sys.path.insert(0, os.environ["ORACLE_PY_DIR"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    # the planted-mistake test runs the oracle pins against a modified copy
    override = os.environ.get("ORACLE_TEST_LIB")
    if override:
        oracle.LIB_PATH = override
    oracle.lib()
    return oracle
