import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_golden(name):
    """Parse a golden text fixture: '#' comments, '[NAME]' headers, rows of numbers.

    Returns a dict of name -> float64 array, or (no headers) one array of rows
    (ragged rows come back as a list of int lists)."""
    blocks, cur, rows = {}, None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                if cur is not None:
                    blocks[cur] = np.array(rows, dtype=np.float64)
                cur, rows = line[1:-1], []
                continue
            rows.append([float(t) for t in line.split()])
    if cur is not None:
        blocks[cur] = np.array(rows, dtype=np.float64)
        return blocks
    return [[int(v) for v in r] for r in rows]


@pytest.fixture
def golden():
    return load_golden
