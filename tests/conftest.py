import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def solver_calls():
    """golden/solver_calls_per_step.txt: scheme -> (solves, roots, RFD
    products by M, printed product total at 5 iterations or None)."""
    rows = {}
    with open(os.path.join(ROOT, "tests", "golden", "solver_calls_per_step.txt")) as fh:
        for line in fh:
            cols = line.split("#")[0].split()
            if cols:
                rows[cols[0]] = (int(cols[1]), int(cols[2]), int(cols[3]), None if cols[4] == "-" else int(cols[4]))
    return rows
