import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import potref
    potref.load()
    return potref


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """How the free-running GPU parity cases were judged (shown even with -q)."""
    try:
        from tests.gpu_common import PARITY_TALLY
    except Exception:
        return
    strict, d1 = PARITY_TALLY["strict"], PARITY_TALLY["def1"]
    if not strict and not d1:
        return
    terminalreporter.write_line(
        f"parity: {len(strict)} free-running cases matched the oracle's decisions (1e-6 element by element), "
        f"{len(d1)} took a near tie the other way and passed the Definition 1 check: {', '.join(d1) or '-'}")
