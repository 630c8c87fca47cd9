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
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    import parity_summary
    rows = parity_summary.lines()
    if rows:
        terminalreporter.write_sep("-", "parity against the oracle, per workload")
        for line in rows:
            terminalreporter.write_line(line)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
