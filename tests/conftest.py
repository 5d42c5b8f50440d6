import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP path through the C-ABI")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """The oracle is plain C; (re)build it once per session so pins never run a stale copy."""
    from oracle import build as ob
    ob.build()
    yield
