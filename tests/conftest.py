import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test (paper statistics over n <= 4096)")


def read_golden(name):
    """Parse a ``key = value`` fixture under tests/golden (``#`` starts a comment)."""
    vals = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (p.strip() for p in line.split("=", 1))
            vals[k] = v
    return vals


@pytest.fixture(scope="session")
def paper_stats():
    return read_golden("paper_statistics.txt")


@pytest.fixture(scope="session")
def error_tables(paper_stats):
    """E_S(n), E_T(n) numerators for n <= 4096 from the C oracle (about 15 s)."""
    from oracle import native
    nmax = int(paper_stats["n_max"])
    return {0: native.error_numerators(nmax, 0), 1: native.error_numerators(nmax, 1)}
