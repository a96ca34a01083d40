"""Affine-normal directions (Section 5) through the C-ABI, against the
oracle's reference route (symbolic derivatives, explicit third-order tensor,
dense tangent solves).  The GPU path contracts third derivatives per
monomial with M = Q_T A^-1 Q_T' and inverts the tangent block by
Gauss-Jordan, so it agrees to rounding, not bitwise: the bound is relative
to |nu| times the tangent block's condition number."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_06575_amd as ph
    ph.lib()
    return ph


def _check(ph, E, C, X, reg, tol=1e-9):
    n = X.shape[1]
    b = ph.batch_from_numpy([0, E.shape[0]], E, C, n=n, max_exp=int(E.max()) if E.size else 0)
    D, gn = ph.affine_normal(b, torch.from_numpy(X).cuda(), reg=reg, check=True)
    D, gn = D.cpu().numpy(), gn.cpu().numpy()
    Do, gno = oracle.affine_normal(E, C, X, reg=reg)
    assert np.allclose(gn, gno, rtol=1e-13, atol=0)
    err = np.abs(D - Do).max(axis=1) / np.abs(Do).max(axis=1)
    say(f"  max relative error {err.max():.3e}")
    assert (err <= tol).all()
    return D


def test_paper_example(ph):
    """Section 5's quartic at x0 with regularization 1e-8: the printed
    direction to its 7 digits, and the oracle's to rounding."""
    g = json.load(open(os.path.join(HERE, "golden", "worked_examples.json")))["W11_affine_example_direction"]
    E = np.array([t[1] for t in g["f"]], np.uint8)
    C = np.array([t[0] for t in g["f"]], float)
    X = np.array([g["x0"]])
    say("affine normal: paper example")
    D = _check(ph, E, C, X, g["regularization"])
    for got, want in zip(D[0], g["d"]):
        assert abs(got - want) <= 0.5e-6 * abs(want) + 1e-22
    b = ph.batch_from_numpy(np.array([0, E.shape[0]], np.int64), E, C, n=4, max_exp=4)
    _, _, info = ph.affine_normal(b, torch.from_numpy(X).cuda(), reg=g["regularization"], info=True)
    assert (info["hv_evals"], info["third_evals"]) == (g["hv_evals"], g["third_evals"])


@pytest.mark.parametrize("n,terms,npts", [(3, 12, 5), (6, 40, 33), (9, 90, 70)])
def test_random_quartics(ph, n, terms, npts):
    """Random quartics with a convex quadratic part, at random points; one
    workgroup per point, several points per launch."""
    rng = W.rng_for(3200 + n)
    E, C = W.random_poly(rng, n, 4, terms)
    E = np.vstack([E, 2 * np.eye(n, dtype=np.uint8)])
    C = np.concatenate([C, 3.0 * np.ones(n)])
    X = rng.uniform(-0.6, 0.6, (npts, n))
    say(f"affine normal: n={n} terms={terms} points={npts}")
    _check(ph, E, C, X, 1e-8)


def test_high_degree_and_pivoting(ph):
    """Degrees up to 8 in four variables (factor lists of several words,
    exponents up to 8) and an indefinite tangent block, so the Gauss-Jordan
    inversion must pivot."""
    rng = W.rng_for(3301)
    n = 4
    E, C = W.random_poly(rng, n, 8, 30)
    E = np.vstack([E, np.array([[2, 0, 0, 0], [0, 2, 0, 0], [0, 0, 2, 0]], np.uint8)])
    C = np.concatenate([C, [2.0, -3.0, 1.5]])
    X = rng.uniform(-0.8, 0.8, (16, n))
    say("affine normal: degree 8, indefinite")
    _check(ph, E, C, X, 0.0, tol=1e-8)


def test_sparse_quartic_n64(ph):
    """A sparse quartic of the paper's timing family (support 3, 4n
    monomials) in n = 64 variables; the oracle's reference route at a few
    points."""
    wl = W.sparse_quartic(seed=W.SEED_BASE + 90, n=64, npts=3)
    say("affine normal: sparse quartic n=64")
    _check(ph, wl.exps, wl.coefs, wl.X, 1e-8, tol=1e-8)


def test_no_points(ph):
    b = ph.batch_from_numpy([0, 1], np.array([[2, 0]], np.uint8), np.array([1.0]), n=2, max_exp=2)
    D, gn = ph.affine_normal(b, torch.zeros((0, 2), dtype=torch.float64, device="cuda"))
    assert D.shape == (0, 2) and gn.shape == (0,)


@pytest.mark.parametrize("n", [65, 70])
def test_register_and_lds_inversion(ph, n):
    """n = 65 is the largest tangent block (64 x 64) inverted in registers;
    n = 70 takes the LDS Gauss-Jordan with row swaps."""
    wl = W.sparse_quartic(seed=W.SEED_BASE + 91 + n, n=n, npts=2)
    say(f"affine normal: sparse quartic n={n}")
    _check(ph, wl.exps, wl.coefs, wl.X, 1e-8, tol=1e-8)


def test_matrix_in_global_memory(ph):
    """n = 130: past the LDS-resident size, the tangent block is inverted in
    the point's Hessian slot of the workspace."""
    wl = W.sparse_quartic(seed=W.SEED_BASE + 221, n=130, npts=1)
    say("affine normal: sparse quartic n=130")
    _check(ph, wl.exps, wl.coefs, wl.X, 1e-8, tol=1e-8)
