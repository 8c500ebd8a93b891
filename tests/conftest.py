import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def golden_blocks(name, rows):
    """Read a numeric fixture from tests/golden and split it into blocks of
    the given row counts."""
    import numpy as np

    data = np.loadtxt(os.path.join(GOLDEN, name), ndmin=2)
    out, r = [], 0
    for n in rows:
        out.append(data[r:r + n])
        r += n
    assert r == data.shape[0], f"{name}: expected {r} rows, found {data.shape[0]}"
    return out
