"""Pins of the oracle's stochastic affine-normal route (Section 5,
MF-logDet-Stochastic) and of its two building blocks, conjugate gradients and
the third-derivative contraction, against what the mathematics fixes:

* conjugate gradients: hand-computed iterates on a 2x2 system, finite
  termination on an SPD system, the stopping rule's minimality, breakdown;
* the contraction D^3 f[u, v, .]: the full third-derivative tensor from
  the symbolic derivatives of the reference route, symmetry in u and v;
* the route itself: probes sqrt(n) times any orthonormal basis of R^n make
  the Hutchinson average the exact trace, so with exact Krylov solves it
  reduces to the exact route; on the quartic of Section 5's example it then
  reproduces the printed direction; with Rademacher probes the direction is
  an unbiased estimate whose covariance has a closed form (the direction is
  affine in the probe average), and the estimate over many probes lies
  within 5 standard deviations of the exact direction in every component."""
import numpy as np

import oracle
import workloads as W


def test_cg_two_by_two_by_hand():
    """A = diag(1, 2), b = (1, 1): alpha_0 = 2/3 gives y_1 = (2/3, 2/3);
    r_1 = (1/3, -1/3), beta_0 = 1/9, p_1 = (4/9, -2/9), alpha_1 = 3/4 gives
    y_2 = (1, 1/2) = A^-1 b."""
    A = np.diag([1.0, 2.0])
    b = np.ones(2)
    y1, k1 = oracle.conjugate_gradients(A, b, 0.0, 1)
    assert k1 == 1 and np.allclose(y1, [2 / 3, 2 / 3], rtol=1e-15, atol=0)
    y2, k2 = oracle.conjugate_gradients(A, b, 0.0, 2)
    assert k2 == 2 and np.allclose(y2, [1.0, 0.5], rtol=1e-15, atol=1e-16)
    # further steps act on a rounding-level residual and leave y in place
    y5, k5 = oracle.conjugate_gradients(A, b, 0.0, 5)
    assert np.allclose(y5, [1.0, 0.5], rtol=1e-15, atol=1e-16)
    # a tolerance stops at the second step
    assert oracle.conjugate_gradients(A, b, 1e-12, 5)[1] == 2


def test_cg_degenerate_inputs():
    A = np.diag([1.0, 2.0, 3.0])
    y, k = oracle.conjugate_gradients(A, np.ones(3), 0.0, 0)
    assert k == 0 and not y.any()
    y, k = oracle.conjugate_gradients(A, np.zeros(3), 0.0, 10)
    assert k == 0 and not y.any()
    # p'Ap = 0 on the first step of an indefinite system: breakdown after
    # one product, nothing taken
    y, k = oracle.conjugate_gradients(np.diag([1.0, -1.0]), np.ones(2), 0.0, 10)
    assert k == 1 and not y.any()


def test_cg_finite_termination_and_stopping_rule():
    rng = W.rng_for(5201)
    m = 7
    B = rng.standard_normal((m, m))
    A = B @ B.T + 0.5 * np.eye(m)
    b = rng.standard_normal(m)
    y, k = oracle.conjugate_gradients(A, b, 0.0, m)
    assert k == m
    assert np.allclose(y, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    tol = 1e-3
    y, k = oracle.conjugate_gradients(A, b, tol, 100)
    assert 1 <= k <= m + 2
    assert np.linalg.norm(b - A @ y) <= tol * np.linalg.norm(b) * (1 + 1e-9)
    y0, _ = oracle.conjugate_gradients(A, b, tol, k - 1)
    assert np.linalg.norm(b - A @ y0) > tol * np.linalg.norm(b)


def _quartic(seed, n, terms):
    rng = W.rng_for(seed)
    E, C = W.random_poly(rng, n, 4, terms)
    E = np.vstack([E, 2 * np.eye(n, dtype=np.uint8)])
    C = np.concatenate([C, 3.0 * np.ones(n)])
    x = rng.uniform(-0.5, 0.5, n)
    return E, C, x, rng


def test_third_contraction_matches_tensor():
    E, C, x, rng = _quartic(5202, 5, 30)
    _, _, T = oracle.derivatives_at(E, C, x, 5)
    u, v = rng.standard_normal(5), rng.standard_normal(5)
    c = oracle.third_contraction(E, C, x, u, v)
    assert np.allclose(c, np.einsum("jkl,j,k->l", T, u, v), rtol=1e-12, atol=1e-12)
    assert np.allclose(c, oracle.third_contraction(E, C, x, v, u), rtol=1e-12, atol=1e-12)
    assert not oracle.third_contraction(E, C, x, np.zeros(5), v).any()


def _golden_poly(entry):
    E = np.array([t[1] for t in entry["f"]], np.uint8)
    C = np.array([t[0] for t in entry["f"]], float)
    return E, C


def test_stochastic_paper_example_with_basis_probes(golden):
    """Probes sqrt(n) e_1 .. sqrt(n) e_n: the tangent probes satisfy
    sum_s z_s z_s' = n Q_T' Q_T = n I, so (1/n) sum_s z_s' M z_s = tr M; with
    conjugate gradients run to termination the route gives the direction
    printed for the example of Section 5."""
    g = golden["W11_affine_example_direction"]
    E, C = _golden_poly(g)
    n = 4
    Z = np.sqrt(n) * np.eye(n)
    D, gn, hv = oracle.affine_normal_stochastic(E, C, np.array([g["x0"]]), Z, g["regularization"], 0.0, 2 * n)
    for got, want in zip(D[0], g["d"]):
        assert abs(got - want) <= 0.5e-6 * abs(want) + 1e-22
    assert abs(gn[0] - g["grad_norm"]) <= 0.5e-6 * g["grad_norm"]
    # one product for H e and, with a zero tolerance, maxit steps for each of
    # the n + 1 solves (none reaches an exactly zero residual)
    assert hv[0] == 1 + (n + 1) * 2 * n


def test_stochastic_reduces_to_exact_route():
    """Any orthonormal basis of R^n, scaled by sqrt(n), as probes."""
    for seed, n, terms in ((5203, 5, 25), (5204, 7, 40)):
        E, C, x, rng = _quartic(seed, n, terms)
        X = np.vstack([x, rng.uniform(-0.5, 0.5, n)])
        R, _ = np.linalg.qr(rng.standard_normal((n, n)))
        Dx, gx = oracle.affine_normal(E, C, X, reg=1e-8)
        for Z in (np.sqrt(n) * np.eye(n), np.sqrt(n) * R.T):
            Ds, gs, hv = oracle.affine_normal_stochastic(E, C, X, Z, 1e-8, 0.0, 3 * n)
            assert np.allclose(Ds, Dx, rtol=1e-9, atol=1e-10)
            assert np.allclose(gs, gx, rtol=1e-14)
        # per-point probes [N, q, n] equal to the shared set give the same
        Z3 = np.broadcast_to(np.sqrt(n) * np.eye(n), (2, n, n))
        D3, _, hv3 = oracle.affine_normal_stochastic(E, C, X, Z3, 1e-8, 0.0, 3 * n)
        assert np.array_equal(D3, oracle.affine_normal_stochastic(E, C, X, np.sqrt(n) * np.eye(n), 1e-8, 0.0, 3 * n)[0])


def test_stochastic_is_unbiased_with_closed_form_covariance():
    """Rademacher probes Z_s in R^n and exact solves.  The route's direction
    is nu = Q_T A^-1 (h - c Q_T' w) - e with c = |g| / (n + 1) and w the probe
    average of w(Z) = D^3 f[M Z, P Z, .] (M = Q_T A^-1 Q_T', P = I - e e'),
    each component w_l(Z) = Z' K_l Z with K_l = M T_l P.  A Rademacher
    quadratic form has mean tr K and covariance Cov(Z'SZ, Z'RZ) =
    2 sum_{i != j} S_ij R_ij for symmetric S, R; so E nu is the exact
    direction and Cov nu = c^2 M Cov(w) M / q."""
    n, q = 5, 3000
    E, C, x, rng = _quartic(5205, n, 25)
    reg = 1e-8
    Z = rng.choice([-1.0, 1.0], size=(q, n))
    Ds, _, _ = oracle.affine_normal_stochastic(E, C, x[None, :], Z, reg, 0.0, 3 * n)
    Dx, _ = oracle.affine_normal(E, C, x[None, :], reg=reg)
    # closed-form covariance from the reference route's derivatives
    g, H, T = oracle.derivatives_at(E, C, x, n)
    Q = oracle.tangent_frame(g)
    QT, e = Q[:, :n - 1], Q[:, n - 1]
    A = QT.T @ H @ QT + reg * np.eye(n - 1)
    M = QT @ np.linalg.solve(A, QT.T)
    P = np.eye(n) - np.outer(e, e)
    S = []
    for l in range(n):
        K = M @ T[:, :, l] @ P
        S.append(0.5 * (K + K.T))
    off = ~np.eye(n, dtype=bool)
    covw = np.array([[2.0 * (S[a] * S[b])[off].sum() for b in range(n)] for a in range(n)])
    c = np.linalg.norm(g) / (n + 1)
    cov = c * c * M @ covw @ M / q
    sd = np.sqrt(np.diag(cov))
    assert (sd > 0).all()
    z = (Ds[0] - Dx[0]) / sd
    assert (np.abs(z) <= 5.0).all(), z
    # and the average is not the exact direction by accident of the seed
    assert np.abs(z).max() > 1e-3
