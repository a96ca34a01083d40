"""Parity at the full workload sizes, in the launch configuration the
benchmark times.  Where the oracle can reproduce a whole output in seconds it
does; otherwise outputs are sampled (points or entries) and compared one by
one, plus properties that hold at any size.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


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


def test_plain_large_full_bitwise(ph):
    """times + simplify of two 5,000-term polynomials in 10 variables
    (25,000,000 raw terms, Gaussian coefficients): every exponent row, the
    order and every coefficient bit agree with the oracle."""
    wl = W.plain_large()
    say("plain large: GPU")
    a = ph.batch_from_numpy([0, 5000], wl.a_exps, wl.a_coefs, n=10, max_exp=8)
    b = ph.batch_from_numpy([0, 5000], wl.b_exps, wl.b_coefs, n=10, max_exp=8)
    rp, E, C = ph.batch_to_numpy(ph.mul(a, b))
    say(f"plain large: {rp[-1]} merged terms; oracle")
    oe, oc = oracle.mul(wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs)
    assert rp[-1] == oe.shape[0]
    assert np.array_equal(E, oe)
    assert C.view(np.uint64).tolist() == oc.view(np.uint64).tolist()


def test_paper_family_pd_cubed(ph):
    """simplify(p_d^3) in five variables (the paper's heavy-simplify family),
    d = 4 and 6: C(3d+5, 5) terms, integer coefficients, bit-exact."""
    import math
    for d in (4, 6):
        e, c = W.all_ones_family(5, d)
        T = e.shape[0]
        say(f"p_{d}^3: base {T}")
        p = ph.batch_from_numpy([0, T], e, c, n=5, max_exp=d)
        sq = ph.mul(p, p)
        sq.max_exp = 2 * d
        cube = ph.mul(sq, p)
        rp, E, C = ph.batch_to_numpy(cube)
        assert rp[-1] == math.comb(3 * d + 5, 5)
        if d == 4:
            oe, oc = oracle.mul(*oracle.mul(e, c, e, c), e, c)
            assert np.array_equal(E, oe) and np.array_equal(C, oc)
        else:
            assert (C >= 1).all() and C.sum() == float(T) ** 3


def test_batch_matrix_full(ph):
    """64 x 64 polynomial matrix, n=20, degree <= 6, log-uniform entry sizes
    in [10, 20000]: the simplify of all 4,096 entries and the whole 64 x 64
    x 20 Jacobian compared bit for bit with the oracle, then the Jacobian's
    evaluation at 4,096 points, every one of the 81,920 polynomials at 16
    sampled points within the per-element bound."""
    from conftest import oracle_over_points
    wl = W.batch_matrix()
    say(f"batch matrix: {wl.row_ptr[-1]} raw terms")
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    s = ph.simplify(b)
    rp, E, C = ph.batch_to_numpy(s)
    say("oracle simplify of all entries")
    orp, oE, oC = oracle.simplify_batch(wl.row_ptr, wl.exps, wl.coefs, n=wl.n)
    assert np.array_equal(rp, orp)
    assert np.array_equal(E, oE)
    assert C.view(np.uint64).tolist() == oC.view(np.uint64).tolist()
    say("jacobian")
    J = ph.jacobian(s)
    jrp, jE, jC = ph.batch_to_numpy(J)
    assert jrp.shape[0] == 4096 * 20 + 1
    say("oracle jacobian of all entries")
    ojrp, ojE, ojC = oracle.jacobian_batch(orp, oE, oC, n=wl.n)
    assert np.array_equal(jrp, ojrp)
    assert np.array_equal(jE, ojE)
    assert jC.view(np.uint64).tolist() == ojC.view(np.uint64).tolist()
    say("jacobian eval")
    Y = ph.eval(J, torch.from_numpy(wl.X).cuda())
    rng = np.random.default_rng(3)
    pts = np.sort(rng.choice(wl.X.shape[0], size=16, replace=False))
    Ys = Y[:, torch.from_numpy(pts).cuda()].cpu().numpy()
    del Y
    say("oracle jacobian eval at 16 points")
    Yo = oracle_over_points(oracle.eval_batch, ojrp, ojE, ojC, wl.X[pts])
    bound = 1e-12 * oracle_over_points(oracle.eval_batch, ojrp, ojE, np.abs(ojC), np.abs(wl.X[pts])) + 1e-300
    assert (np.abs(Ys - Yo) <= bound).all()


def test_dense_shared_full_sampled(ph):
    """4,096 polynomials over 46,376 monomials at 65,536 points: FP64 MFMA
    and split BF16 (S=5) against the oracle on all polynomials at 8 points."""
    wl = W.dense_shared()
    basis = torch.from_numpy(wl.basis).cuda()
    C = torch.from_numpy(wl.C).cuda()
    X = torch.from_numpy(wl.X).cuda()
    pts = np.array([0, 1, 777, 20000, 40000, 65000, 65534, 65535])
    say("dense oracle sample")
    Yo = oracle.eval_dense(wl.basis, wl.C, wl.X[pts])
    A = oracle.eval_dense(wl.basis, np.abs(wl.C), np.abs(wl.X[pts]))
    for prec, S, tol in ((ph.POLY_FP64, 5, 1e-12), (ph.POLY_SPLIT_BF16, 5, 1e-10)):
        say(f"dense prec={prec}")
        Y = ph.eval_dense(basis, C, X, prec=prec, nslices=S)
        Ys = Y[:, torch.from_numpy(pts).cuda()].cpu().numpy()
        err = np.abs(Ys - Yo) / A
        say(f"  max condition-scaled error {err.max():.3e}")
        assert err.max() <= tol
        rel = np.abs(Ys - Yo) / np.abs(Yo)
        assert np.median(rel) <= tol
        del Y


def test_dense_backward_full_sampled(ph):
    """Reverse mode of the 4,096 x 46,376 x 65,536 contraction with a
    cotangent that is zero except at 8 points.  References from the oracle:
    dC[p][k] = sum over the 8 points of gY[p][pt] v_k(x_pt), with v_k the
    oracle's values of the one-term polynomials x^{e_k}; dX at each of those
    points is the oracle's gradient of the single polynomial
    sum_p gY[p][pt] f_p (coefficients gY[:, pt] C, a NumPy product).  Every
    element within 1e-12 times the same sums over absolute values; dX rows
    of the other points exactly zero."""
    wl = W.dense_shared()
    P, K, N = wl.C.shape[0], wl.basis.shape[0], wl.X.shape[0]
    pts = np.array([0, 1, 777, 20000, 40000, 65000, 65534, 65535])
    g8 = W.rng_for(4020).standard_normal((P, pts.size))
    gY = torch.zeros((P, N), dtype=torch.float64, device="cuda")
    gY[:, torch.from_numpy(pts).cuda()] = torch.from_numpy(g8).cuda()
    say("dense backward full size")
    dC, dX = ph.eval_dense_backward(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                                    torch.from_numpy(wl.X).cuda(), gY)
    dC, dX = dC.cpu().numpy(), dX.cpu().numpy()
    del gY
    say("references over 8 points")
    X8 = wl.X[pts]
    one = np.arange(K + 1, dtype=np.int64)
    V = oracle.eval_batch(one, wl.basis, np.ones(K), X8)              # [K, 8] monomial values
    Va = oracle.eval_batch(one, wl.basis, np.ones(K), np.abs(X8))
    assert (np.abs(dC - g8 @ V.T) <= 1e-12 * (np.abs(g8) @ Va.T) + 1e-300).all()
    for i, pt in enumerate(pts):
        cw = g8[:, i] @ wl.C                                            # coefficients of sum_p gY f_p
        ca = np.abs(g8[:, i]) @ np.abs(wl.C)
        G = oracle.grad_batch([0, K], wl.basis, cw, X8[i:i + 1])[0, 0]
        Ga = oracle.grad_batch([0, K], wl.basis, ca, np.abs(X8[i:i + 1]))[0, 0]
        assert (np.abs(dX[pt] - G) <= 1e-12 * Ga + 1e-12 * np.abs(G) + 1e-300).all()
    rest = np.ones(N, bool)
    rest[pts] = False
    assert not dX[rest].any()


def test_dense_backward_split_full_sampled(ph):
    """Split reverse mode of the 4,096 x 46,376 x 65,536 contraction (5
    digits) with a dense N(0,1) cotangent.  dC: 16 rows x 64 monomials against
    the oracle's monomial values over all 65,536 points (dC[p][k] = gY[p] .
    v_k, a NumPy dot product), each within 1e-10 of sum_pt |gY v_k|; the FP64
    kernel's entries there within 1e-12.  dX (16 chunks of W): 8 points
    against the oracle's gradient of sum_p gY[p][pt] f_p (coefficients
    gY[:, pt] C, a NumPy product), each within 1e-10 of the same sums over
    absolute values."""
    wl = W.dense_shared()
    P, K, N = wl.C.shape[0], wl.basis.shape[0], wl.X.shape[0]
    gY = W.rng_for(4030).standard_normal((P, N))
    say("split dC full size")
    args = [torch.from_numpy(a).cuda() for a in (wl.basis, wl.C, wl.X, gY)]
    dC, dX = ph.eval_dense_backward(*args, prec=ph.POLY_SPLIT_BF16, nslices=5)
    pts = np.array([0, 1, 4095, 4096, 30000, 65000, 65534, 65535])
    dX = dX[torch.from_numpy(pts).cuda()].cpu().numpy()
    rows = np.sort(W.rng_for(4031).choice(P, 16, replace=False))
    cols = np.sort(W.rng_for(4032).choice(K, 64, replace=False))
    dCs = dC[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy()
    del dC
    dC64 = ph.eval_dense_backward(*args, want_dX=False)[0]
    dC64s = dC64[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy()
    del dC64, args
    say("references over all points for 64 monomials")
    one = np.arange(cols.size + 1, dtype=np.int64)
    V = oracle.eval_batch(one, wl.basis[cols], np.ones(cols.size), wl.X)            # [64, N]
    Va = oracle.eval_batch(one, wl.basis[cols], np.ones(cols.size), np.abs(wl.X))
    ref = gY[rows] @ V.T
    A = np.abs(gY[rows]) @ Va.T
    err = np.abs(dCs - ref) / A
    say(f"  dC max condition-scaled error {err.max():.3e}")
    assert err.max() <= 1e-10
    assert (np.abs(dC64s - ref) <= 1e-12 * A).all()
    say("dX references at 8 points")
    for i, pt in enumerate(pts):
        cw = gY[:, pt] @ wl.C
        ca = np.abs(gY[:, pt]) @ np.abs(wl.C)
        G = oracle.grad_batch([0, K], wl.basis, cw, wl.X[pt:pt + 1])[0, 0]
        Ga = oracle.grad_batch([0, K], wl.basis, ca, np.abs(wl.X[pt:pt + 1]))[0, 0]
        e = np.abs(dX[i] - G) / Ga
        say(f"  dX point {pt}: max condition-scaled error {e.max():.3e}")
        assert (e <= 1e-10).all()


def test_quartic_full_sampled(ph):
    """Random quartic in 100 variables with 100,000 terms at 8,192 points:
    value, gradient (reverse-mode kernel with unit cotangent and poly_grad)
    and Hessian (poly_hess) against the oracle's symbolic derivatives at 64
    sampled points, every element within 1e-12 times the same sum over
    absolute values; Hessian symmetric bit for bit; gradient against central
    differences of the GPU's own evaluation."""
    from conftest import oracle_over_points
    wl = W.quartic()
    b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=100, max_exp=4)
    X = torch.from_numpy(wl.X).cuda()
    pts = np.unique(np.concatenate([[0, 8191], np.random.default_rng(5).choice(8192, size=62, replace=False)]))
    rp = np.array([0, wl.exps.shape[0]], np.int64)
    Xs, aC, aXs = wl.X[pts], np.abs(wl.coefs), np.abs(wl.X[pts])
    say("quartic eval")
    Y = ph.eval(b, X).cpu().numpy()[0]
    yo = oracle.eval_batch(rp, wl.exps, wl.coefs, Xs)[0]
    assert (np.abs(Y[pts] - yo) <= 1e-12 * oracle.eval_batch(rp, wl.exps, aC, aXs)[0] + 1e-300).all()
    say("quartic backward (gradient)")
    dX, dC = ph.eval_backward(b, X, torch.ones((1, X.shape[0]), dtype=torch.float64, device="cuda"), check=True)
    G = ph.grad(b, X, check=True).cpu().numpy()[0]
    say("oracle gradient at 64 points")
    Go = oracle_over_points(oracle.grad_batch, rp, wl.exps, wl.coefs, Xs)[0]
    gtol = 1e-12 * oracle_over_points(oracle.grad_batch, rp, wl.exps, aC, aXs)[0] + 1e-300
    assert (np.abs(dX.cpu().numpy()[pts] - Go) <= gtol).all()
    assert (np.abs(G[pts] - Go) <= gtol).all()
    say("quartic hessian")
    H = ph.hess(b, X[torch.from_numpy(pts).cuda()].contiguous(), check=True).cpu().numpy()[0]
    say("oracle hessian at 64 points")
    Ho = oracle_over_points(oracle.hess_batch, rp, wl.exps, wl.coefs, Xs)[0]
    assert (np.abs(H - Ho) <= 1e-12 * oracle_over_points(oracle.hess_batch, rp, wl.exps, aC, aXs)[0] + 1e-300).all()
    assert np.array_equal(H, np.swapaxes(H, 1, 2))
    say("finite differences")
    h = 1e-6
    Xp = X.clone()
    Xm = X.clone()
    Xp[:, 7] += h
    Xm[:, 7] -= h
    fd = (ph.eval(b, Xp) - ph.eval(b, Xm)).cpu().numpy()[0] / (2 * h)
    assert np.allclose(fd, G[:, 7], rtol=1e-6, atol=1e-6)


def test_quartic_integer_full_bitwise(ph):
    """The same shape with integer coefficients in [-9, 9] at integer points in
    {-2..2}^100: every value, gradient and Hessian entry is an integer below
    2^53, so any summation order is exact and the GPU must agree with the
    oracle bit for bit: values at all 8,192 points, gradients (from both
    poly_grad and the reverse-mode kernel) at 2,048 of them, Hessians at 256."""
    from conftest import oracle_over_points
    wl = W.quartic()
    C = W.rng_for(W.SEED_BASE + 55).integers(-9, 10, size=wl.coefs.shape[0]).astype(np.float64)
    Xn = W.integer_points(W.SEED_BASE + 56, 8192, 100, -2, 2)
    rp = np.array([0, wl.exps.shape[0]], np.int64)
    b = ph.batch_from_numpy(rp, wl.exps, C, n=100, max_exp=4)
    X = torch.from_numpy(Xn).cuda()
    say("integer quartic: eval")
    Y = ph.eval(b, X).cpu().numpy()
    say("integer quartic: oracle eval at 8,192 points")
    assert np.array_equal(Y, oracle_over_points(oracle.eval_batch, rp, wl.exps, C, Xn))
    say("integer quartic: gradient (poly_grad, reverse mode)")
    G = ph.grad(b, X, check=True).cpu().numpy()
    dX, _ = ph.eval_backward(b, X, torch.ones((1, 8192), dtype=torch.float64, device="cuda"), want_dC=False,
                             check=True)
    dX = dX.cpu().numpy()
    sel = np.arange(0, 8192, 4)
    say("integer quartic: oracle gradient at 2,048 points")
    Go = oracle_over_points(oracle.grad_batch, rp, wl.exps, C, Xn[sel])
    assert np.array_equal(G[:, sel], Go)
    assert np.array_equal(dX[sel], Go[0])
    sel = np.arange(0, 8192, 32)
    say("integer quartic: hessian at 256 points")
    H = ph.hess(b, X[torch.from_numpy(sel).cuda()].contiguous(), check=True).cpu().numpy()
    assert np.array_equal(H, oracle_over_points(oracle.hess_batch, rp, wl.exps, C, Xn[sel]))
