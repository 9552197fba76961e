import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size case, minutes of CPU time")


@pytest.fixture(scope="session")
def dpdlib():
    """The built library (built in place first if it is missing)."""
    import paper_2205_05158_amd as D
    from paper_2205_05158_amd import build as B
    if not os.path.exists(D.LIB_PATH):
        B.build()
    return D.lib()
