import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle():
    """The CPU oracle's ctypes front end (built on first use)."""
    from oracle import build_oracle, pyoracle
    if not os.path.exists(pyoracle.LIB_PATH):
        build_oracle.build()
    return pyoracle
