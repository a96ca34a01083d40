"""Pins for the CPU oracle: worked examples the paper prints, closed forms,
exact identities, brute force on tiny inputs.  No GPU involved.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a transposed index, a wrong order, an unstable merge) fails at
least one test here.
"""
import math

import numpy as np
import pytest
from scipy import signal

import oracle
import workloads as W
from conftest import as_termset, poly_from_json


def _poly(g, key):
    return poly_from_json(g[key], g["n"])


# --------------------------------------------------------------- worked examples

def test_w1_canonical_order(golden):
    g = golden["W1_scalar_workflow"]
    e, c = _poly(g, "input")
    oe, oc = oracle.simplify(e, c)
    xe, xc = _poly(g, "simplified")
    assert np.array_equal(oe, xe) and np.array_equal(oc, xc)
    assert int(oe.astype(int).sum(axis=1).max()) == g["degree"]


def test_w2_diff_grad_eval(golden):
    g = golden["W2_differentiation"]
    n = g["n"]
    e, c = _poly(g, "input")
    de, dc = oracle.diff(e, c, 0)
    # diff keeps storage order; simplify gives the printed (canonical) order
    se, sc = oracle.simplify(de, dc)
    xe, xc = poly_from_json(g["diff_x1"], n)
    assert np.array_equal(se, xe) and np.array_equal(sc, xc)
    for j, expect in enumerate(g["jacobian"]):
        je, jc = oracle.diff(e, c, j)
        ee, ec = poly_from_json(expect, n)
        assert as_termset(*oracle.simplify(je, jc)) == as_termset(ee, ec)
    x = np.array([g["point"]], dtype=np.float64)
    assert oracle.eval_points(e, c, x)[0] == g["value"]
    G = oracle.grad_batch([0, len(c)], e, c, x)[0, 0]
    assert G.tolist() == [7.0, 2.0, -1.0]          # [3x1^2 + 2x2, 2x1, -1] at (1,2,3)
    H = oracle.hess_batch([0, len(c)], e, c, x)[0, 0]
    assert H.tolist() == [[6.0, 2.0, 0.0], [2.0, 0.0, 0.0], [0.0, 0.0, 0.0]]


def test_w3_trace_merge(golden):
    g = golden["W3_trace"]
    n = g["n"]
    parts = [poly_from_json(t, n) for t in g["diagonal"]]
    e = np.vstack([p[0] for p in parts])
    c = np.concatenate([p[1] for p in parts])
    oe, oc = oracle.simplify(e, c)
    assert as_termset(oe, oc) == as_termset(*_poly(g, "trace"))


def test_w4_monolist_count(golden):
    g = golden["W4_monolist"]
    assert W.basis(g["n"], g["d"]).shape[0] == g["count"] == math.comb(g["n"] + g["d"], g["d"])


def test_w5_simplify_order(golden):
    g = golden["W5_mixed_simplify"]
    pe, pc = _poly(g, "p")
    qe, qc = _poly(g, "q")
    oe, oc = oracle.simplify(np.vstack([pe, qe]), np.concatenate([pc, qc]))
    xe, xc = _poly(g, "simplified")
    assert np.array_equal(oe, xe) and np.array_equal(oc, xc)


def test_w6_matrix_ops(golden):
    g = golden["W6_matrix_ops"]
    n = g["n"]
    A = [poly_from_json(t, n) for t in g["A"]]
    sq = [oracle.mul(a[0], a[1], a[0], a[1]) for a in A]
    for got, exp in zip(sq, g["elem_square"]):
        assert as_termset(*got) == as_termset(*poly_from_json(exp, n))
    assert sq[2][0].shape[0] == 0                    # 0 .* 0 is the structural zero
    # matrix square: C_ij = simplify(sum_k A_ik A_kj), 2x2 row-major
    for i in range(2):
        for j in range(2):
            prods = [oracle.mul(*A[i * 2 + k], *A[k * 2 + j]) for k in range(2)]
            e = np.vstack([p[0] for p in prods])
            c = np.concatenate([p[1] for p in prods])
            got = oracle.simplify(e, c, n=n)
            assert as_termset(*got) == as_termset(*poly_from_json(g["matrix_square"][i * 2 + j], n))
    # sum(A,1): column sums
    for j in range(2):
        e = np.vstack([A[j][0], A[2 + j][0]])
        c = np.concatenate([A[j][1], A[2 + j][1]])
        assert as_termset(*oracle.simplify(e, c, n=n)) == as_termset(*poly_from_json(g["sum_dim1"][j], n))
    # prod(A,2): row products
    for i in range(2):
        got = oracle.mul(*A[i * 2], *A[i * 2 + 1])
        assert as_termset(*got) == as_termset(*poly_from_json(g["prod_dim2"][i], n))


def test_w8_substitution_expansion(golden):
    g = golden["W8_substitution"]
    n = g["n"]
    ue, uc = _poly(g, "u")
    assert uc.tolist() == [3.0, 5.0]                 # constructor keeps the caller's order
    s = _poly(g, "z1_plus_1")
    sq = oracle.mul(*s, *s)                          # (z1+1)^2
    three = (np.zeros((1, n), np.uint8), np.array([3.0]))
    t1 = oracle.mul(*three, *sq)
    e = np.vstack([t1[0], np.array([[0, 1]], np.uint8)])
    c = np.concatenate([t1[1], [5.0]])
    assert as_termset(*oracle.simplify(e, c)) == as_termset(*_poly(g, "result"))


def test_w9_quadratic_form(golden):
    g = golden["W9_quadratic_form"]
    n = g["n"]
    Q = g["Q"]
    b = [poly_from_json(t, n) for t in g["b"]]
    es, cs = [], []
    for i in range(2):
        for j in range(2):
            qe, qc = oracle.mul(*b[i], *b[j])
            es.append(qe)
            cs.append(qc * Q[i][j])
    got = oracle.simplify(np.vstack(es), np.concatenate(cs))
    assert as_termset(*got) == as_termset(*_poly(g, "qf"))


def test_w11_gradient_norm(golden):
    g = golden["W11_affine_example_gradient"]
    e, c = _poly(g, "f")
    G = oracle.grad_batch([0, len(c)], e, c, np.array([g["x0"]]))[0, 0]
    assert round(float(np.linalg.norm(G)), 6) == g["grad_norm"]


def test_xy_square(golden):
    g = golden["XY_square"]
    p = _poly(g, "p")
    oe, oc = oracle.mul(*p, *p)
    xe, xc = _poly(g, "square")
    assert np.array_equal(oe, xe) and np.array_equal(oc, xc)


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n,d", [(2, 2), (3, 4), (4, 5), (5, 3), (6, 4)])
def test_multinomial_closed_form(n, d):
    """(x1+...+xn)^d has C(n+d-1, d) terms with coefficients d!/prod(a_i!)."""
    lin = (np.eye(n, dtype=np.uint8), np.ones(n))
    acc = (np.zeros((1, n), np.uint8), np.ones(1))
    for _ in range(d):
        acc = oracle.mul(*acc, *lin)
    e, c = acc
    assert e.shape[0] == math.comb(n + d - 1, d)
    for row, coef in zip(e.astype(int).tolist(), c.tolist()):
        assert sum(row) == d
        expect = math.factorial(d)
        for a in row:
            expect //= math.factorial(a)
        assert coef == expect
    # ascending canonical order
    assert all(tuple(e[i]) < tuple(e[i + 1]) for i in range(e.shape[0] - 1))


@pytest.mark.parametrize("d", [2, 3])
def test_pd_cubed_closed_form(golden, d):
    """simplify(p_d^3) in five variables (Section 6.3): C(3d+5, 5) terms; the
    coefficient of x^g counts triples (a, b, c), |a|,|b|,|c| <= d, a+b+c = g.
    The counts come from a dense 5-D convolution (no sorting, no merging)."""
    n = 5
    e, c = W.all_ones_family(n, d)
    assert e.shape[0] == golden["PD_family"]["base_counts"][str(d)]
    sq = oracle.mul(e, c, e, c)
    cube = oracle.mul(*sq, e, c)
    assert cube[0].shape[0] == math.comb(3 * d + 5, 5)
    ind = np.zeros((d + 1,) * n)
    for row in e.astype(int):
        ind[tuple(row)] = 1.0
    dense = signal.convolve(signal.convolve(ind, ind, method="direct"), ind, method="direct")
    dense = np.rint(dense).astype(np.int64)
    nz = np.argwhere(dense > 0)
    assert nz.shape[0] == cube[0].shape[0]
    for row, coef in zip(cube[0].astype(int), cube[1]):
        assert dense[tuple(row)] == coef


# ------------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(12))
def test_simplify_matches_brute_force(seed):
    rng = W.rng_for(1000 + seed)
    n = int(rng.integers(1, 6))
    d = int(rng.integers(0, 5))
    t = int(rng.integers(0, 60))
    e, c = W.random_poly(rng, n, d, t, integer=bool(seed % 2))
    if seed % 3 == 0 and t:
        c[rng.integers(0, t, size=max(1, t // 5))] = 0.0
    for tol in (0.0, 0.5):
        oe, oc = oracle.simplify(e, c, tol, n=n)
        be, bc = oracle.brute_simplify(e.reshape(-1, n), c, tol)
        assert np.array_equal(oe, be)
        assert oc.view(np.uint64).tolist() == bc.view(np.uint64).tolist()


@pytest.mark.parametrize("seed", range(8))
def test_mul_matches_brute_force(seed):
    rng = W.rng_for(2000 + seed)
    n = int(rng.integers(1, 5))
    a = W.random_poly(rng, n, 3, int(rng.integers(0, 12)), integer=bool(seed % 2))
    b = W.random_poly(rng, n, 3, int(rng.integers(0, 12)), integer=bool(seed % 2))
    # brute force: nested loops over a Python dict
    raw_e, raw_c = [], []
    for i in range(a[0].shape[0]):
        for j in range(b[0].shape[0]):
            raw_e.append([int(x) + int(y) for x, y in zip(a[0][i], b[0][j])])
            raw_c.append(float(a[1][i]) * float(b[1][j]))
    be, bc = oracle.brute_simplify(np.array(raw_e, dtype=np.uint8).reshape(-1, n), np.array(raw_c))
    oe, oc = oracle.mul(*a, *b, n=n)
    assert np.array_equal(oe, be)
    assert oc.view(np.uint64).tolist() == bc.view(np.uint64).tolist()


def test_zero_rule_and_nan():
    e = np.array([[1], [1], [2], [3], [3], [4]], dtype=np.uint8)
    c = np.array([1.0, -1.0, 1e-3, np.nan, 1.0, -0.0])
    oe, oc = oracle.simplify(e, c, 0.0)
    assert oe.ravel().tolist() == [2, 3]             # 1-1 = 0 and -0.0 dropped; NaN kept
    assert oc[0] == 1e-3 and np.isnan(oc[1])
    oe, oc = oracle.simplify(e, c, 1e-3)
    assert oe.ravel().tolist() == [3]                # |1e-3| <= tol is dropped


# ------------------------------------------------------------------- identities

def test_mul_coefficient_sum_invariant():
    wl = W.plain_small()
    oe, oc = oracle.mul(wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs)
    assert oc.sum() == wl.a_coefs.sum() * wl.b_coefs.sum()
    assert oe.shape[0] <= 1820 and (oc != 0).all()


@pytest.mark.parametrize("seed", range(4))
def test_eval_product_identity_bitwise(seed):
    """eval(p*q) == eval(p)*eval(q) exactly at small integer points with
    integer coefficients (every intermediate stays below 2^53)."""
    rng = W.rng_for(3000 + seed)
    n = 3
    p = W.random_poly(rng, n, 4, 15)
    q = W.random_poly(rng, n, 4, 15)
    pq = oracle.mul(*p, *q)
    X = W.integer_points(3100 + seed, 32, n)
    yp = oracle.eval_points(*p, X)
    yq = oracle.eval_points(*q, X)
    ypq = oracle.eval_points(*pq, X)
    assert np.array_equal(ypq, yp * yq)


def test_eval_constants_and_empty():
    X = np.array([[0.0, 0.0], [2.0, -1.0]])
    empty = (np.zeros((0, 2), np.uint8), np.zeros(0))
    assert oracle.eval_points(*empty, X).tolist() == [0.0, 0.0]
    const = (np.zeros((1, 2), np.uint8), np.array([-4.5]))
    assert oracle.eval_points(*const, X).tolist() == [-4.5, -4.5]
    zero_pow = (np.array([[0, 3]], np.uint8), np.array([2.0]))   # 0^0 = 1 at x1 = 0
    assert oracle.eval_points(*zero_pow, X).tolist() == [0.0, -2.0]


def test_eval_dense_against_numpy_power():
    b = W.basis(3, 4)
    rng = W.rng_for(77)
    C = rng.integers(-5, 6, size=(4, b.shape[0])).astype(np.float64)
    X = W.integer_points(78, 10, 3, -2, 2)
    V = np.prod(X[None, :, :] ** b.astype(np.float64)[:, None, :], axis=2)   # [K, N]
    assert np.array_equal(oracle.eval_dense(b, C, X), C @ V)
    Yld, A = oracle.eval_dense_ld(b, C, X)
    assert np.array_equal(Yld, C @ V)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_euler_identities_bitwise(d):
    n = 4
    e, c = W.homogeneous(40 + d, n, d, 25)
    X = W.integer_points(50 + d, 16, n, -3, 3)
    rp = [0, e.shape[0]]
    f = oracle.eval_batch(rp, e, c, X)[0]
    G = oracle.grad_batch(rp, e, c, X)[0]
    H = oracle.hess_batch(rp, e, c, X)[0]
    assert np.array_equal((G * X).sum(axis=1), d * f)
    assert np.array_equal(np.einsum("pjk,pk->pj", H, X), (d - 1) * G)


def test_hessian_symmetry_and_second_jacobian():
    rng = W.rng_for(91)
    n = 5
    e, c = W.random_poly(rng, n, 5, 40, integer=False)
    X = W.points(92, 8, n)
    H = oracle.hess_batch([0, e.shape[0]], e, c, X)[0]
    assert np.array_equal(H, np.swapaxes(H, 1, 2))
    # with integer coefficients the Hessian equals jacobian(jacobian(p)) exactly
    ei, ci = W.random_poly(rng, n, 5, 40, integer=True)
    Hi = oracle.hess_batch([0, ei.shape[0]], ei, ci, X)[0]
    for j in range(n):
        dj = oracle.diff(ei, ci, j)
        for k in range(n):
            djk = oracle.diff(*dj, k)
            assert np.array_equal(oracle.eval_points(*djk, X), Hi[:, j, k])


def test_gradient_and_hessian_vs_finite_differences():
    rng = W.rng_for(93)
    n = 4
    e, c = W.random_poly(rng, n, 4, 30, integer=False)
    X = W.points(94, 6, n, -0.9, 0.9)
    rp = [0, e.shape[0]]
    G = oracle.grad_batch(rp, e, c, X)[0]
    H = oracle.hess_batch(rp, e, c, X)[0]
    h = 1e-5
    for j in range(n):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, j] += h
        Xm[:, j] -= h
        fd = (oracle.eval_batch(rp, e, c, Xp)[0] - oracle.eval_batch(rp, e, c, Xm)[0]) / (2 * h)
        assert np.allclose(fd, G[:, j], rtol=1e-7, atol=1e-7)
        fdg = (oracle.grad_batch(rp, e, c, Xp)[0] - oracle.grad_batch(rp, e, c, Xm)[0]) / (2 * h)
        assert np.allclose(fdg, H[:, :, j], rtol=1e-6, atol=1e-6)


def test_diff_product_rule_bitwise():
    rng = W.rng_for(95)
    n = 3
    p = W.random_poly(rng, n, 3, 10)
    q = W.random_poly(rng, n, 3, 10)
    X = W.integer_points(96, 12, n)
    pq = oracle.mul(*p, *q)
    for j in range(n):
        lhs = oracle.eval_points(*oracle.diff(*pq, j), X)
        rhs = oracle.eval_points(*oracle.diff(*p, j), X) * oracle.eval_points(*q, X) \
            + oracle.eval_points(*p, X) * oracle.eval_points(*oracle.diff(*q, j), X)
        assert np.array_equal(lhs, rhs)


def test_eval_backward_pins():
    rng = W.rng_for(97)
    n = 3
    polys = [W.random_poly(rng, n, 3, k) for k in (7, 0, 12)]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.integer_points(98, 9, n, -2, 2)
    P = len(polys)
    # gY = 1: dX is the sum of gradients; dC_t is the sum over points of v_t
    dX, dC = oracle.eval_backward(rp, E, C, X, np.ones((P, X.shape[0])))
    G = oracle.grad_batch(rp, E, C, X)
    assert np.array_equal(dX, G.sum(axis=0))
    V = np.prod(X[None, :, :] ** E.astype(np.float64)[:, None, :], axis=2)
    assert np.array_equal(dC, V.sum(axis=1))
    # linearity in C: <gY, Y(C + dC') - Y(C)> = <dC, dC'>  (integers: exact)
    gY = rng.integers(-3, 4, size=(P, X.shape[0])).astype(np.float64)
    _, dC = oracle.eval_backward(rp, E, C, X, gY, want_dX=False)
    delta = rng.integers(-3, 4, size=C.shape[0]).astype(np.float64)
    Y0 = oracle.eval_batch(rp, E, C, X)
    Y1 = oracle.eval_batch(rp, E, C + delta, X)
    assert (gY * (Y1 - Y0)).sum() == (dC * delta).sum()


def test_eval_backward_dx_vs_finite_differences():
    rng = W.rng_for(99)
    n = 3
    polys = [W.random_poly(rng, n, 4, 9, integer=False) for _ in range(3)]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.points(100, 5, n)
    gY = rng.standard_normal((3, 5))
    dX, _ = oracle.eval_backward(rp, E, C, X, gY, want_dC=False)
    h = 1e-6
    for pt in range(5):
        for j in range(n):
            Xp, Xm = X.copy(), X.copy()
            Xp[pt, j] += h
            Xm[pt, j] -= h
            fd = ((oracle.eval_batch(rp, E, C, Xp) - oracle.eval_batch(rp, E, C, Xm)) * gY).sum() / (2 * h)
            assert abs(fd - dX[pt, j]) <= 1e-7 * (1 + abs(fd))


def test_eval_backward2_vs_finite_differences_of_eval_backward():
    """The second-order reverse mode is the gradient of L = <w, dC> + <u, dX>
    with (dC, dX) from eval_backward: central differences of L in every
    point coordinate, every cotangent entry and every coefficient."""
    rng = W.rng_for(131)
    n = 3
    polys = [W.random_poly(rng, n, 4, 8, integer=False) for _ in range(2)]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.points(132, 4, n)
    gY = rng.standard_normal((2, 4))
    u = rng.standard_normal((4, n))
    w = rng.standard_normal(C.shape[0])
    ggY, ggX, ggC = oracle.eval_backward2(rp, E, C, X, gY, u, w)

    def L(C_, X_, gY_):
        dX, dC = oracle.eval_backward(rp, E, C_, X_, gY_)
        return (w * dC).sum() + (u * dX).sum()

    h = 1e-6
    for pt in range(4):
        for j in range(n):
            Xp, Xm = X.copy(), X.copy()
            Xp[pt, j] += h
            Xm[pt, j] -= h
            fd = (L(C, Xp, gY) - L(C, Xm, gY)) / (2 * h)
            assert abs(fd - ggX[pt, j]) <= 1e-7 * (1 + abs(fd))
    for p in range(2):
        for pt in range(4):
            gp, gm = gY.copy(), gY.copy()
            gp[p, pt] += h
            gm[p, pt] -= h
            fd = (L(C, X, gp) - L(C, X, gm)) / (2 * h)
            assert abs(fd - ggY[p, pt]) <= 1e-7 * (1 + abs(fd))
    for t in range(C.shape[0]):
        cp, cm = C.copy(), C.copy()
        cp[t] += h
        cm[t] -= h
        fd = (L(cp, X, gY) - L(cm, X, gY)) / (2 * h)
        assert abs(fd - ggC[t]) <= 1e-7 * (1 + abs(fd))


def test_eval_backward2_closed_form():
    """f = 3 x1^2 x2 - x2 x3^3 at (x1, x2, x3) = (1, 2, -1), gY = 2, u = (1, 0, 1),
    w = (1, 1): Hess f = [[6 x2, 6 x1, 0], [6 x1, 0, -3 x3^2], [0, -3 x3^2, -6 x2 x3]]
    = [[12, 6, 0], [6, 0, -3], [0, -3, 12]], so ggX = 2 (H u + grad(x1^2 x2 + x2 x3^3))
    = 2 ([12, 3, 12] + [2 x1 x2, x1^2 + x3^3, 3 x2 x3^2]) = 2 ([12, 3, 12] + [4, 0, 6]);
    ggY = grad f . u + (x1^2 x2 + x2 x3^3) = (6 x1 x2 - 3 x2 x3^2) + 0 = 6;
    ggC = 2 (grad(x1^2 x2) . u, grad(x2 x3^3) . u) = 2 (2 x1 x2, 3 x2 x3^2) = (8, 12)."""
    E = np.array([[2, 1, 0], [0, 1, 3]], np.uint8)
    C = np.array([3.0, -1.0])
    X = np.array([[1.0, 2.0, -1.0]])
    ggY, ggX, ggC = oracle.eval_backward2([0, 2], E, C, X, np.array([[2.0]]), np.array([[1.0, 0.0, 1.0]]),
                                          np.array([1.0, 1.0]))
    assert np.array_equal(ggX, np.array([[32.0, 6.0, 36.0]]))
    assert np.array_equal(ggY, np.array([[6.0]]))
    assert np.array_equal(ggC, np.array([8.0, 12.0]))


def test_fp64_eval_within_error_bound_of_long_double():
    wl = W.quartic(seed=5, n=12, terms=1500, npts=64)
    rp = [0, wl.exps.shape[0]]
    y = oracle.eval_batch(rp, wl.exps, wl.coefs, wl.X)[0]
    yl, A = oracle.eval_batch_ld(rp, wl.exps, wl.coefs, wl.X)
    # a-priori bound for a T-term recursive sum of products of <= 5 factors
    T = wl.exps.shape[0]
    bound = (T + 6) * 2.0 ** -53 * A[0]
    assert (np.abs(y - yl[0]) <= bound).all()


def test_jacobian_batch_layout():
    rng = W.rng_for(101)
    n = 3
    polys = [W.random_poly(rng, n, 3, k) for k in (5, 0, 8)]
    rp, E, C = W.csr_from_list(polys, n)
    jrp, jE, jC = oracle.jacobian_batch(rp, E, C)
    assert jrp.shape[0] == 3 * n + 1
    for p in range(3):
        for j in range(n):
            k = p * n + j
            de, dc = oracle.diff(*polys[p], j)
            assert np.array_equal(jE[jrp[k]:jrp[k + 1]], de)
            assert np.array_equal(jC[jrp[k]:jrp[k + 1]], dc)


# ------------------------------------------------------------- affine normal

def _golden_poly(entry):
    E = np.array([t[1] for t in entry["f"]], np.uint8)
    C = np.array([t[0] for t in entry["f"]], float)
    return E, C


def test_affine_normal_paper_example(golden):
    """Section 5's printed direction (7 significant digits) at x0 with
    regularization 1e-8.  The third component, -1.01e-9, exists only through
    the regularized tangent solves, and the first, second and fourth depend on
    the |g| / (n + 1) weight of the log-det correction, so the example pins
    both readings."""
    g = golden["W11_affine_example_direction"]
    E, C = _golden_poly(g)
    D, gn = oracle.affine_normal(E, C, np.array([g["x0"]]), reg=g["regularization"])
    for got, want in zip(D[0], g["d"]):
        assert abs(got - want) <= 0.5e-6 * abs(want) + 1e-22
    assert abs(gn[0] - g["grad_norm"]) <= 0.5e-6 * g["grad_norm"]


def _random_quartic(seed, n, terms):
    rng = W.rng_for(seed)
    E, C = W.random_poly(rng, n, 4, terms)
    # a convex quadratic part keeps the tangent block well conditioned
    E = np.vstack([E, 2 * np.eye(n, dtype=np.uint8)])
    C = np.concatenate([C, 3.0 * np.ones(n)])
    x = rng.uniform(-0.5, 0.5, n)
    return E, C, x, rng


def test_affine_normal_quadric_closed_form():
    """For a quadratic f the third derivatives vanish and the direction is
    -H^-1 e / (e' H^-1 e) (its affine normal line passes through the
    centre), computed here from the full Hessian with no tangent frame."""
    rng = W.rng_for(3101)
    n = 6
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)          # f = 1/2 x'Ax + b'x
    b = rng.standard_normal(n)
    E, C = [], []
    for j in range(n):
        for k in range(j, n):
            e = np.zeros(n, np.uint8)
            e[j] += 1
            e[k] += 1
            E.append(e)
            C.append(A[j, j] / 2 if j == k else A[j, k])
        e = np.zeros(n, np.uint8)
        e[j] = 1
        E.append(e)
        C.append(b[j])
    x = rng.uniform(-1, 1, n)
    D, _ = oracle.affine_normal(np.array(E), np.array(C), x[None, :], reg=0.0)
    g = A @ x + b
    e = g / np.linalg.norm(g)
    u = np.linalg.solve(A, e)
    assert np.allclose(D[0], -u / (e @ u), rtol=1e-11, atol=1e-12)


def test_affine_normal_frame_invariance():
    """Any orthonormal completion of e gives the same direction."""
    E, C, x, rng = _random_quartic(3102, 5, 25)
    g, H, T = oracle.derivatives_at(E, C, x, 5)
    Q = oracle.tangent_frame(g)
    R, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    Q2 = np.column_stack([Q[:, :4] @ R, Q[:, 4]])
    nu1, _ = oracle.affine_normal_from_derivatives(g, H, T, 0.0, Q)
    nu2, _ = oracle.affine_normal_from_derivatives(g, H, T, 0.0, Q2)
    assert np.allclose(nu1, nu2, rtol=1e-10, atol=1e-12)


def test_affine_normal_equiaffine_covariance():
    """For y = A x with det A = 1, the derivatives of f(A^-1 y) are the
    tensors of f transformed by A^-1 in every index, and the affine normal
    there is A times the affine normal of f (the normalisation e'nu = -1 only
    rescales it): a transposed frame or a wrong contraction breaks this."""
    E, C, x, rng = _random_quartic(3103, 5, 25)
    g, H, T = oracle.derivatives_at(E, C, x, 5)
    nu, _ = oracle.affine_normal_from_derivatives(g, H, T, 0.0)
    A = rng.standard_normal((5, 5))
    A /= np.sign(np.linalg.det(A)) * abs(np.linalg.det(A)) ** 0.2
    Ai = np.linalg.inv(A)
    g2, H2 = Ai.T @ g, Ai.T @ H @ Ai
    T2 = np.einsum("jkl,ja,kb,lc->abc", T, Ai, Ai, Ai)
    nu2, _ = oracle.affine_normal_from_derivatives(g2, H2, T2, 0.0)
    r = nu2 / (A @ nu)
    assert (r > 0).all() and np.ptp(r) <= 1e-9 * r.mean()


# ------------------------------------------------------- polynomial matrices

def _mat(polys, n):
    rp, E, C = W.csr_from_list(polys, n)
    return rp, E, C


def test_mtimes_paper_matrix_square(golden):
    """Section 3.3: A = [x1, 1; 0, x2], A^2 = [x1^2, x1 + x2; 0, x2^2]."""
    g = golden["W6_matrix_ops"]
    n = g["n"]
    A = [poly_from_json(t, n) for t in g["A"]]
    rp, E, C = _mat(A, n)
    orp, oe, oc = oracle.mtimes(rp, E, C, rp, E, C, 2, 2, 2, n=n)
    for q in range(4):
        got = (oe[orp[q]:orp[q + 1]], oc[orp[q]:orp[q + 1]])
        assert as_termset(*got) == as_termset(*poly_from_json(g["matrix_square"][q], n))
    assert orp[3] == orp[2]                          # the (2,1) entry is the structural zero


def test_mtimes_identity_and_scalar_case():
    """A I = A bitwise for simplified entries (products by 1 are exact), and
    a 1 x 1 product is the entrywise times."""
    rng = W.rng_for(3401)
    n = 3
    A = [oracle.simplify(*W.random_poly(rng, n, 3, 12, integer=False), n=n) for _ in range(6)]   # 2 x 3
    one = (np.zeros((1, n), np.uint8), np.array([1.0]))
    zero = (np.zeros((0, n), np.uint8), np.zeros(0))
    Id = [one if i == j else zero for i in range(3) for j in range(3)]
    arp, ae, ac = _mat(A, n)
    irp, ie, ic = _mat(Id, n)
    orp, oe, oc = oracle.mtimes(arp, ae, ac, irp, ie, ic, 2, 3, 3, n=n)
    assert np.array_equal(orp, arp) and np.array_equal(oe, ae)
    assert oc.view(np.uint64).tolist() == ac.view(np.uint64).tolist()
    p, q = A[0], A[1]
    _, e1, c1 = oracle.mtimes([0, p[0].shape[0]], p[0], p[1], [0, q[0].shape[0]], q[0], q[1], 1, 1, 1, n=n)
    e2, c2 = oracle.mul(p[0], p[1], q[0], q[1], n=n)
    assert np.array_equal(e1, e2) and np.array_equal(c1, c2)


def test_mtimes_associative_on_integers():
    """(A B) C = A (B C) exactly when every coefficient is a small integer."""
    rng = W.rng_for(3402)
    n = 3
    A = [W.random_poly(rng, n, 2, 5) for _ in range(2 * 3)]
    B = [W.random_poly(rng, n, 2, 5) for _ in range(3 * 2)]
    Cm = [W.random_poly(rng, n, 2, 5) for _ in range(2 * 2)]
    a, b, c = _mat(A, n), _mat(B, n), _mat(Cm, n)
    ab = oracle.mtimes(*a, *b, 2, 3, 2, n=n)
    left = oracle.mtimes(*ab, *c, 2, 2, 2, n=n)
    bc = oracle.mtimes(*b, *c, 3, 2, 2, n=n)
    right = oracle.mtimes(*a, *bc, 2, 3, 2, n=n)
    assert all(np.array_equal(x, y) for x, y in zip(left, right))


def test_msum_mprod_paper_example(golden):
    """Section 3.3: sum(A, 1) = [x1, 1 + x2] and prod(A, 2) = [x1; 0] for
    A = [x1, 1; 0, x2]."""
    g = golden["W6_matrix_ops"]
    n = g["n"]
    rp, E, C = _mat([poly_from_json(t, n) for t in g["A"]], n)
    srp, se, sc = oracle.msum(rp, E, C, 2, 2, 1, n=n)
    for q in range(2):
        assert as_termset(se[srp[q]:srp[q + 1]], sc[srp[q]:srp[q + 1]]) == \
            as_termset(*poly_from_json(g["sum_dim1"][q], n))
    prp, pe, pc = oracle.mprod(rp, E, C, 2, 2, 2, n=n)
    assert as_termset(pe[prp[0]:prp[1]], pc[prp[0]:prp[1]]) == as_termset(*poly_from_json(g["prod_dim2"][0], n))
    assert prp[2] == prp[1]                          # 0 * x2 is the structural zero


@pytest.mark.parametrize("dim", [1, 2])
def test_msum_mprod_eval_identities(dim):
    """At integer points with small integer coefficients every value is exact:
    eval(sum(A, dim)) is the sum and eval(prod(A, dim)) the product of the
    entries' values along dim, taken independently of the oracle's simplify
    (values of the unsimplified entries)."""
    rng = W.rng_for(3410 + dim)
    n, R, Cc = 3, 3, 4
    A = [W.random_poly(rng, n, 2, int(rng.integers(0, 6))) for _ in range(R * Cc)]
    rp, E, C = _mat(A, n)
    X = rng.integers(-2, 3, size=(5, n)).astype(np.float64)
    vals = np.array([[sum(c * np.prod(x ** e.astype(np.float64)) for e, c in zip(*A[q])) for x in X]
                     for q in range(R * Cc)]).reshape(R, Cc, -1)
    srp, se, sc = oracle.msum(rp, E, C, R, Cc, dim, n=n)
    prp, pe, pc = oracle.mprod(rp, E, C, R, Cc, dim, n=n)
    want_s = vals.sum(axis=dim - 1)
    want_p = vals.prod(axis=dim - 1)
    got_s = oracle.eval_batch(srp, se, sc, X)
    got_p = oracle.eval_batch(prp, pe, pc, X)
    assert np.array_equal(got_s.reshape(want_s.shape), want_s)
    assert np.array_equal(got_p.reshape(want_p.shape), want_p)


def test_msum_mprod_degenerate():
    """Empty dimension: sum gives structural zeros, prod the constant 1; a
    dimension of length one gives the simplified entries themselves."""
    n = 2
    rp, E, C = _mat([], n)
    srp, _, _ = oracle.msum(rp, E, C, 3, 0, 2, n=n)
    assert srp.tolist() == [0, 0, 0, 0]
    prp, pe, pc = oracle.mprod(rp, E, C, 3, 0, 2, n=n)
    assert prp.tolist() == [0, 1, 2, 3] and not pe.any() and pc.tolist() == [1.0, 1.0, 1.0]
    rng = W.rng_for(3420)
    A = [W.random_poly(rng, n, 3, 8, integer=False) for _ in range(3)]
    rp, E, C = _mat(A, n)
    want = oracle.simplify_batch(rp, E, C, n=n)
    for f in (oracle.msum, oracle.mprod):
        got = f(rp, E, C, 3, 1, 2, n=n)
        assert all(np.array_equal(x, y) for x, y in zip(got, want))


def test_subs_paper_example(golden):
    """Section 3.4: u = 3 x1^2 + 5 x2, u(z1 + 1, z2) = 3 + 6 z1 + 3 z1^2 + 5 z2."""
    g = golden["W8_substitution"]
    n = g["n"]
    ue, uc = poly_from_json(g["u"], n)
    q = [poly_from_json(g["z1_plus_1"], n), (np.array([[0, 1]], np.uint8), np.array([1.0]))]
    rp, E, C = _mat(q, n)
    e, c = oracle.subs(ue, uc, rp, E, C, n)
    assert as_termset(e, c) == as_termset(*poly_from_json(g["result"], n))


def test_subs_identity_and_values():
    """Substituting x_i for x_i gives simplify(p) bitwise; at small integer
    points with integer coefficients, subs(p, q)(z) = p(q_1(z), ..., q_n(z))
    exactly (values taken directly, not through the oracle)."""
    rng = W.rng_for(3430)
    n, m = 3, 2
    pe, pc = W.random_poly(rng, n, 3, 12, integer=False)
    ids = [(np.eye(n, dtype=np.uint8)[i:i + 1], np.ones(1)) for i in range(n)]
    rp, E, C = _mat(ids, n)
    e, c = oracle.subs(pe, pc, rp, E, C, n)
    se, sc = oracle.simplify(pe, pc, n=n)
    assert np.array_equal(e, se) and c.view(np.uint64).tolist() == sc.view(np.uint64).tolist()
    pe, pc = W.random_poly(rng, n, 3, 8)
    q = [W.random_poly(rng, m, 2, 3) for _ in range(n)]
    rp, E, C = _mat(q, m)
    e, c = oracle.subs(pe, pc, rp, E, C, m)
    Z = rng.integers(-2, 3, size=(4, m)).astype(np.float64)

    def val(ee, cc, x):
        return sum(ci * np.prod(x ** ei.astype(np.float64)) for ei, ci in zip(ee, cc))

    for z in Z:
        qz = np.array([val(*qi, z) for qi in q])
        assert val(e, c, z) == val(pe, pc, qz)
