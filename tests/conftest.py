import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libpw")
    config.addinivalue_line("markers", "slow: long-running CPU test")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def read_golden(name):
    """Rows of a golden fixture: whitespace-separated ints, last column an arithmetic
    expression in sqrt/pi/integers (evaluated with nothing else in scope)."""
    import math
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            ints = tuple(int(p) for p in parts[:-1])
            val = eval(parts[-1], {"__builtins__": {}}, {"sqrt": math.sqrt, "pi": math.pi})
            rows.append((ints, float(val)))
    return rows


@pytest.fixture
def golden():
    return read_golden
