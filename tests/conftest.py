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


def read_golden(name):
    """Numeric blocks of a golden fixture; '# ...' lines separate blocks."""
    blocks, cur = [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            s = line.strip()
            if not s:
                continue
            if s.startswith("#"):
                if cur:
                    blocks.append(np.array(cur, dtype=np.float64))
                    cur = []
                continue
            cur.append([float(t) for t in s.split()])
    if cur:
        blocks.append(np.array(cur, dtype=np.float64))
    return blocks


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle
