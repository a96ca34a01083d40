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
    in [10, 20000]: one persistent simplify launch, then the 64 x 64 x 20
    Jacobian, then its evaluation at 4,096 points (sampled entries/points
    against the oracle)."""
    wl = W.batch_matrix()
    say(f"batch matrix: {wl.row_ptr[-1]} raw terms")
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    s = ph.simplify(b)
    rp, E, C = ph.batch_to_numpy(s)
    rng = np.random.default_rng(3)
    entries = np.sort(rng.choice(4096, size=256, replace=False))
    entries = np.unique(np.concatenate([entries, [int(np.argmax(np.diff(wl.row_ptr)))]]))
    for p in entries:
        lo, hi = wl.row_ptr[p], wl.row_ptr[p + 1]
        oe, oc = oracle.simplify(wl.exps[lo:hi], wl.coefs[lo:hi])
        assert np.array_equal(E[rp[p]:rp[p + 1]], oe)
        assert C[rp[p]:rp[p + 1]].view(np.uint64).tolist() == oc.view(np.uint64).tolist()
    say("jacobian")
    J = ph.jacobian(s)
    jrp, jE, jC = ph.batch_to_numpy(J)
    assert jrp.shape[0] == 4096 * 20 + 1
    for p in entries[:64]:
        for j in range(20):
            de, dc = oracle.diff(E[rp[p]:rp[p + 1]], C[rp[p]:rp[p + 1]], j)
            k = p * 20 + j
            assert np.array_equal(jE[jrp[k]:jrp[k + 1]], de)
            assert np.array_equal(jC[jrp[k]:jrp[k + 1]], dc)
    say("jacobian eval")
    Y = ph.eval(J, torch.from_numpy(wl.X).cuda())
    pts = np.sort(rng.choice(wl.X.shape[0], size=16, replace=False))
    Ys = Y[:, torch.from_numpy(pts).cuda()].cpu().numpy()
    sel = np.array([p * 20 + j for p in entries[:32] for j in range(20)])
    for k in sel:
        e_, c_ = jE[jrp[k]:jrp[k + 1]], jC[jrp[k]:jrp[k + 1]]
        yo = oracle.eval_points(e_, c_, wl.X[pts])
        bound = 1e-12 * oracle.eval_points(e_, np.abs(c_), np.abs(wl.X[pts])) + 1e-300
        assert (np.abs(Ys[k] - yo) <= bound).all()


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


def test_quartic_full_sampled(ph):
    """Random quartic in 100 variables with 100,000 terms at 8,192 points:
    value, gradient (reverse-mode kernel with unit cotangent and poly_grad)
    and Hessian (poly_hess) against the oracle's symbolic derivatives on
    sampled points; Hessian symmetric bit for bit; gradient against central
    differences of the GPU's own evaluation."""
    wl = W.quartic()
    b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=100, max_exp=4)
    X = torch.from_numpy(wl.X).cuda()
    pts = np.array([0, 5, 4096, 8191])
    rp = [0, wl.exps.shape[0]]
    say("quartic eval")
    Y = ph.eval(b, X).cpu().numpy()[0]
    yo = oracle.eval_batch(rp, wl.exps, wl.coefs, wl.X[pts])[0]
    assert np.allclose(Y[pts], yo, rtol=0, atol=1e-12 * oracle.eval_batch(rp, wl.exps, np.abs(wl.coefs), np.abs(wl.X[pts]))[0].max())
    say("quartic backward (gradient)")
    dX, dC = ph.eval_backward(b, X, torch.ones((1, X.shape[0]), dtype=torch.float64, device="cuda"), check=True)
    G = ph.grad(b, X, check=True).cpu().numpy()[0]
    Go = oracle.grad_batch(rp, wl.exps, wl.coefs, wl.X[pts])[0]
    scale = np.abs(Go).max()
    assert np.abs(dX.cpu().numpy()[pts] - Go).max() <= 1e-11 * scale
    assert np.abs(G[pts] - Go).max() <= 1e-11 * scale
    say("quartic hessian")
    H = ph.hess(b, X[torch.from_numpy(pts).cuda()].contiguous(), check=True).cpu().numpy()[0]
    Ho = oracle.hess_batch(rp, wl.exps, wl.coefs, wl.X[pts])[0]
    assert np.abs(H - Ho).max() <= 1e-11 * np.abs(Ho).max()
    assert np.array_equal(H, np.swapaxes(H, 1, 2))
    say("finite differences")
    h = 1e-6
    Xp = X.clone()
    Xm = X.clone()
    Xp[:, 7] += h
    Xm[:, 7] -= h
    fd = (ph.eval(b, Xp) - ph.eval(b, Xm)).cpu().numpy()[0] / (2 * h)
    assert np.allclose(fd, G[:, 7], rtol=1e-6, atol=1e-6)
