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


def oracle_over_points(fn, row_ptr, exps, coefs, X, nthreads=None):
    """fn(row_ptr, exps, coefs, X_chunk) (an oracle evaluation returning
    [P, pts, ...]) over row chunks of X in a thread pool.  The oracle's C
    routines run with the GIL released, so the chunks run in parallel; every
    output element is computed exactly as in a single call."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    nthreads = nthreads or min(16, os.cpu_count() or 1)
    X = np.ascontiguousarray(X)
    chunks = [c for c in np.array_split(np.arange(X.shape[0]), nthreads) if c.size]
    with ThreadPoolExecutor(max_workers=len(chunks)) as ex:
        parts = list(ex.map(lambda c: fn(row_ptr, exps, coefs, X[c[0]:c[-1] + 1]), chunks))
    return np.concatenate(parts, axis=1)


def monomial_values(basis, X):
    """V [K, N]: the oracle's values of the one-term polynomials x^{e_k}."""
    import numpy as np
    import oracle
    K = basis.shape[0]
    return oracle.eval_batch(np.arange(K + 1, dtype=np.int64), basis, np.ones(K), X)


def block_scaled_reference(V, gY, pb=128):
    """sum over 128-point blocks b of max_b |gY_p| sum_b |v_k| + sum_b |gY_p|
    max_b |v_k|: the quantity the split dC's truncation error is proportional
    to (the digits of both operands are relative to their block's largest
    magnitude)."""
    import numpy as np
    aV, aG = np.abs(V), np.abs(gY)
    ref = np.zeros((gY.shape[0], V.shape[0]))
    for p0 in range(0, gY.shape[1], pb):
        g, v = aG[:, p0:p0 + pb], aV[:, p0:p0 + pb]
        ref += g.max(1)[:, None] * v.sum(1)[None, :] + g.sum(1)[:, None] * v.max(1)[None, :]
    return ref


def split_dx_reference(basis, C, X, gY, pb=128):
    """sum_k refW[k][pt] |d v_k / d x_j (x_pt)| with refW[k][pt] the
    block-scaled reference of W = C^T gY over 128-polynomial blocks b,
    max_b |C_k| sum_b |gY_pt| + sum_b |C_k| max_b |gY_pt|: the quantity the
    split dX's truncation error is proportional to (the error of each W
    entry, carried by the exact derivative factors)."""
    import numpy as np
    import oracle
    K = basis.shape[0]
    D = np.abs(oracle.grad_batch(np.arange(K + 1, dtype=np.int64), basis, np.ones(K), X))   # [K, N, n]
    aC, aG = np.abs(C), np.abs(gY)
    refW = np.zeros((K, X.shape[0]))
    for p0 in range(0, C.shape[0], pb):
        c, g = aC[p0:p0 + pb], aG[p0:p0 + pb]
        refW += c.max(0)[:, None] * g.sum(0)[None, :] + c.sum(0)[:, None] * g.max(0)[None, :]
    return np.einsum("kp,kpj->pj", refW, D)
