"""poly_affine_normal_stochastic (Section 5, MF-logDet-Stochastic) against
the oracle's stochastic route on the same probes.

Both sides run conjugate gradients with the same stopping rule on the same
tangent problems, so they take the same number of steps (checked through the
Hessian-vector product counts) and differ only by rounding: the oracle works
in the coordinates of a tangent frame with the formed tangent block, the
kernel in R^n on e-perp with matrix-free products and LDS atomics.  Each
conjugate-gradient solve amplifies a relative rounding difference by about
the condition number of its tangent block (below 1e3 on these workloads),
so the directions are held to 1e-9 relative to their norm.  Points are
drawn in the locally convex regime Section 5 works in, where the tangent
blocks are positive definite (support-3 families at |x_i| <= 0.35, support-2
at |x_i| <= 0.25: condition numbers below 10 on these seeds); on indefinite
blocks the truncated iterates are far more sensitive to rounding.

Cases: the example of Section 5 with basis probes (the printed direction),
the accuracy preset of the paper's accuracy tables (q = 64, 80 steps) on a
sparse quartic in 6 variables with 17 monomials, the speed preset of its
crossover study (q = 1, reg 5e-4, tol 2e-2, 6 steps) on support-2 quartics
with m = 3n, probe counts that make every group shape of the kernel (one
probe per 256, 128, 64 and 4 threads, a partial last batch), per-point
probes, the reduction to the exact route, and the error paths."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
RTOL = 1e-9


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


def run(ph, E, C, X, Z, reg, tol, maxit):
    n = E.shape[1]
    b = ph.batch_from_numpy(np.array([0, E.shape[0]], np.int64), E, C, n=n, max_exp=int(E.max()))
    D, gn, hv = ph.affine_normal_stochastic(b, torch.from_numpy(X).cuda(), torch.from_numpy(np.ascontiguousarray(Z)).cuda(),
                                            reg=reg, tol=tol, maxit=maxit, check=True)
    return D.cpu().numpy(), gn.cpu().numpy(), hv.cpu().numpy()


def compare(ph, E, C, X, Z, reg, tol, maxit, label):
    say(f"{label}: n={E.shape[1]}, {E.shape[0]} terms, {X.shape[0]} points, q={Z.shape[-2]}, "
        f"reg={reg}, tol={tol}, maxit={maxit}")
    D, gn, hv = run(ph, E, C, X, Z, reg, tol, maxit)
    Do, go, hvo = oracle.affine_normal_stochastic(E, C, X, Z, reg, tol, maxit)
    err = np.abs(D - Do).max(axis=1) / np.linalg.norm(Do, axis=1)
    say(f"  max relative error {err.max():.2e}, products per point {hv.min()}..{hv.max()}")
    assert np.isfinite(D).all()
    assert (err <= RTOL).all(), err.max()
    assert np.allclose(gn, go, rtol=1e-13)
    assert np.array_equal(hv, hvo)
    return D, hv


def test_paper_example_basis_probes(ph, golden):
    g = golden["W11_affine_example_direction"]
    E = np.array([t[1] for t in g["f"]], np.uint8)
    C = np.array([t[0] for t in g["f"]], float)
    n = 4
    Z = np.sqrt(n) * np.eye(n)
    D, hv = compare(ph, E, C, np.array([g["x0"]]), Z, g["regularization"], 0.0, 2 * n, "Section 5 example")
    for got, want in zip(D[0], g["d"]):
        assert abs(got - want) <= 0.5e-6 * abs(want) + 1e-22
    assert hv[0] == 1 + (n + 1) * 2 * n


def test_accuracy_preset_six_variables(ph):
    """q = 64 Rademacher probes, 80 steps, tolerance 1e-4, reg 1e-8."""
    wl = W.sparse_quartic(seed=5301, n=6, npts=48, m=11)
    assert wl.exps.shape[0] == 17
    Z = W.rng_for(5302).choice([-1.0, 1.0], size=(64, 6))
    compare(ph, wl.exps, wl.coefs, wl.X * 0.5, Z, 1e-8, 1e-4, 80, "accuracy preset")


@pytest.mark.parametrize("n", [80, 120])
def test_speed_preset_crossover_family(ph, n):
    """Support-2 quartics with m = 3n; q = 1, reg 5e-4, tol 2e-2, 6 steps."""
    wl = W.sparse_quartic(seed=5310 + n, n=n, npts=24, support=2)
    Z = W.rng_for(5311 + n).choice([-1.0, 1.0], size=(1, n))
    compare(ph, wl.exps, wl.coefs, wl.X * 0.25, Z, 5e-4, 2e-2, 6, "speed preset")


@pytest.mark.parametrize("n,q", [(9, 1), (9, 2), (9, 3), (9, 64), (9, 100), (200, 8)])
def test_group_shapes(ph, n, q):
    """q = 1, 2, 3 (4 slots), 64 and 100 (a full and a partial batch);
    n = 200 with 8 probes runs 4 slots at a time (the LDS budget)."""
    wl = W.sparse_quartic(seed=5320 + q, n=n, npts=6 if n > 50 else 40)
    Z = W.rng_for(5321 + q).choice([-1.0, 1.0], size=(q, n))
    compare(ph, wl.exps, wl.coefs, wl.X * 0.35, Z, 1e-6, 1e-6, 40, f"group shapes q={q}")


def test_per_point_probes(ph):
    wl = W.sparse_quartic(seed=5330, n=7, npts=30)
    Z = W.rng_for(5331).standard_normal((30, 5, 7))
    compare(ph, wl.exps, wl.coefs, wl.X * 0.35, Z, 1e-6, 1e-8, 40, "per-point probes")


def test_basis_probes_reduce_to_exact_route(ph):
    """sqrt(n) times an orthonormal basis as probes and solves run to
    termination: the GPU's exact route gives the same directions."""
    n = 8
    wl = W.sparse_quartic(seed=5340, n=n, npts=32)
    X = wl.X * 0.35
    R, _ = np.linalg.qr(W.rng_for(5341).standard_normal((n, n)))
    D, _, _ = run(ph, wl.exps, wl.coefs, X, np.sqrt(n) * R.T, 1e-8, 0.0, 3 * n)
    b = ph.batch_from_numpy(np.array([0, wl.exps.shape[0]], np.int64), wl.exps, wl.coefs, n=n, max_exp=2)
    Dx, _ = ph.affine_normal(b, torch.from_numpy(X).cuda(), reg=1e-8, check=True)
    Dx = Dx.cpu().numpy()
    err = np.abs(D - Dx).max(axis=1) / np.linalg.norm(Dx, axis=1)
    say(f"basis probes vs exact route: max relative difference {err.max():.2e}")
    assert (err <= RTOL).all()


def test_degenerate_solves(ph):
    """Two variables (a one-dimensional tangent space), no Krylov steps at all
    (maxit = 0: every solve returns 0 and the direction is -e), and a single
    point with a single probe."""
    E = np.array([[4, 0], [2, 2], [0, 2], [1, 0], [0, 0]], np.uint8)
    C = np.array([1.0, 0.5, 2.0, 0.3, 1.0])
    X = np.array([[0.3, -0.2], [0.1, 0.4], [-0.25, 0.15]])
    Z = np.array([[1.0, -1.0], [1.0, 1.0]])
    # a tolerance, not 0: in one dimension the oracle's residual can vanish
    # exactly after the first step while the kernel's (in R^2) keeps a
    # rounding-level remainder, and a zero tolerance would count the extra steps
    D, hv = compare(ph, E, C, X, Z, 1e-8, 1e-12, 3, "n = 2")
    assert (hv == 4).all()   # H e, then one step for each of the three solves
    D, hv = compare(ph, E, C, X, Z, 1e-8, 1e-6, 0, "no Krylov steps")
    assert (hv == 1).all()
    compare(ph, E, C, X[:1], Z[:1], 1e-8, 1e-12, 5, "one point, one probe")


def test_errors_and_empty(ph):
    wl = W.sparse_quartic(seed=5350, n=5, npts=4)
    b = ph.batch_from_numpy(np.array([0, wl.exps.shape[0]], np.int64), wl.exps, wl.coefs, n=5, max_exp=2)
    Z = torch.ones((2, 5), dtype=torch.float64, device="cuda")
    D, gn, hv = ph.affine_normal_stochastic(b, torch.empty((0, 5), dtype=torch.float64, device="cuda"), Z)
    assert D.shape == (0, 5) and gn.shape == (0,)
    with pytest.raises(ph.PolyError):
        ph.affine_normal_stochastic(b, torch.from_numpy(wl.X).cuda(), Z, tol=-1.0)
    # a term of total degree 13 is beyond the factor-list encoding
    E = np.vstack([wl.exps, np.array([[13, 0, 0, 0, 0]], np.uint8)])
    C = np.concatenate([wl.coefs, [1.0]])
    b2 = ph.batch_from_numpy(np.array([0, E.shape[0]], np.int64), E, C, n=5, max_exp=13)
    say("degree-13 term: device status")
    with pytest.raises(ph.PolyError) as ex:
        ph.affine_normal_stochastic(b2, torch.from_numpy(wl.X).cuda(), Z, check=True)
    assert ex.value.code == 6
