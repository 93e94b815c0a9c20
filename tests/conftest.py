import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """Parse a tests/golden fixture: 'key: values' lines, '#' comments.
    Clause lists are DIMACS literals separated by '|'."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            s = line.strip()
            if not s or s.startswith("#"):
                continue
            key, val = s.split(":", 1)
            key, val = key.strip(), val.strip()
            if key.endswith("clauses"):
                out[key] = [[int(t) for t in c.split()] for c in val.split("|")]
            else:
                out[key] = [float(t) for t in val.split()]
    return out


@pytest.fixture
def golden():
    return read_golden
