import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """The oracle is test infrastructure: build it once per session if missing."""
    lib = os.path.join(ROOT, "oracle", "libvlct_ref.so")
    src = os.path.join(ROOT, "oracle", "vlct_ref.c")
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        from oracle import build
        build.build()
    yield
