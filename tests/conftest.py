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


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Tracks the oracle flags as ill-conditioned are excluded from the parity
    counts; list them (always, not only with -s)."""
    try:
        from tests.gpu_util import FLAGGED
    except Exception:
        return
    if not FLAGGED:
        return
    terminalreporter.section("oracle-flagged tracks (listed, not counted)")
    for what, n, first in FLAGGED:
        terminalreporter.write_line(f"{what}: {n} tracks, first ids {first}")
