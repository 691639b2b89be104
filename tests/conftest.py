import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X, gfx950)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    from oracle import build as obuild
    if not os.path.exists(oracle.LIB_PATH):
        obuild.build()
    return oracle.default()
