import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs a gfx950 GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build
    if not (os.path.exists(build.LIB) and os.path.exists(build.LIB_OMP)):
        build.build()
    yield
