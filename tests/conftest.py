import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def golden():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "worked_examples.json")) as f:
        return json.load(f)


def poly_from_json(terms, n):
    """[[coef, [e1..en]], ...] -> (uint8 [T, n], float64 [T])."""
    import numpy as np
    if not terms:
        return np.zeros((0, n), dtype=np.uint8), np.zeros(0)
    e = np.array([t[1] for t in terms], dtype=np.uint8).reshape(-1, n)
    c = np.array([t[0] for t in terms], dtype=np.float64)
    return e, c


def as_termset(e, c):
    return sorted((tuple(int(v) for v in row), float(x)) for row, x in zip(e.tolist(), c.tolist()))
