import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.lib()


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """How the fp64 parity comparisons of the session went (bit for bit, or
    within the tolerance, and how often only the cancellation clause of the
    tolerance held)."""
    import sys as _sys
    gu = _sys.modules.get("gpu_util")
    if gu is not None and gu.FP64_TALLY["comparisons"]:
        terminalreporter.write_line(f"fp64 parity: {gu.FP64_TALLY}")
