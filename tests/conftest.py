import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def piclib():
    """The built HIP library (built here only if nothing is built yet)."""
    from paper_2104_00642_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2104_00642_amd import build
        build.build()
    return _lib.lib()
