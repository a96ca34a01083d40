"""Run-to-run determinism: the same call twice on the same inputs gives the
same bits.  Keys, counts and order are fixed by construction everywhere;
coefficients and values are fixed wherever the summation order is (merges
sum runs left to right in one lane, evaluations sum terms in order, the MFMA
contractions accumulate in a fixed order).  Paths that add into LDS with
atomics (the affine-normal kernels' third-derivative contractions, the fused
derivative kernels, the dense reverse mode's dX) are checked to agree to
rounding instead."""
import sys

import numpy as np
import pytest
import torch

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
    old = ph.tune_get("simplify_wide_min")
    yield ph
    ph.tune_set("simplify_wide_min", old)


def bits(x):
    a = x.cpu().numpy() if torch.is_tensor(x) else np.asarray(x)
    return np.ascontiguousarray(a).view(np.uint8)


def same_batch(ph, a, b):
    ra, rb = ph.batch_to_numpy(a), ph.batch_to_numpy(b)
    return all(np.array_equal(bits(x), bits(y)) for x, y in zip(ra, rb))


def test_times_and_simplify_paths(ph):
    wl = W.plain_large(seed=W.SEED_BASE + 90, terms=2000)
    rp = [0, 2000]
    a = ph.batch_from_numpy(rp, wl.a_exps, wl.a_coefs, n=wl.n, max_exp=wl.max_exp)
    b = ph.batch_from_numpy(rp, wl.b_exps, wl.b_coefs, n=wl.n, max_exp=wl.max_exp)
    say("times, one large pair (radix sort path)")
    assert same_batch(ph, ph.mul(a, b), ph.mul(a, b))
    bm = W.batch_matrix(seed=W.SEED_BASE + 91, entries=64, tmin=10, tmax=4000, npts=0)
    m = ph.batch_from_numpy(bm.row_ptr, bm.exps, bm.coefs, n=bm.n, max_exp=bm.max_exp)
    say("times, batch (bucket path)")
    assert same_batch(ph, ph.mul(m, m), ph.mul(m, m))
    for wide in (1 << 62, 1):
        ph.tune_set("simplify_wide_min", wide)
        say(f"simplify ({'per entry' if wide > 1 else 'device-wide'})")
        assert same_batch(ph, ph.simplify(m), ph.simplify(m))
    wk = W.batch_matrix(seed=W.SEED_BASE + 92, entries=40, n=40, tmin=10, tmax=3000, npts=0)
    k = ph.batch_from_numpy(wk.row_ptr, wk.exps, wk.coefs, n=wk.n, max_exp=wk.max_exp)
    say("simplify over key words")
    assert same_batch(ph, ph.simplify(k), ph.simplify(k))


def test_evaluation_paths(ph):
    wl = W.batch_matrix(seed=W.SEED_BASE + 93, entries=16, n=8, d=5, tmin=10, tmax=2000, npts=700)
    b = ph.simplify(ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp))
    X = torch.from_numpy(wl.X).cuda()
    for name, fn in (("eval", ph.eval), ("grad", ph.grad), ("hess", ph.hess)):
        say(name)
        assert np.array_equal(bits(fn(b, X)), bits(fn(b, X)))
    gY = torch.from_numpy(W.rng_for(94).standard_normal((b.npolys, X.shape[0]))).cuda()
    say("reverse mode")
    dX1, dC1 = ph.eval_backward(b, X, gY)
    dX2, dC2 = ph.eval_backward(b, X, gY)
    assert np.array_equal(bits(dX1), bits(dX2)) and np.array_equal(bits(dC1), bits(dC2))


def test_dense_paths(ph):
    wl = W.dense_shared(seed=W.SEED_BASE + 95, P=90, N=300, n=8, d=4, K=330)
    basis, C, X = (torch.from_numpy(x).cuda() for x in (wl.basis, wl.C, wl.X))
    for prec in (ph.POLY_FP64, ph.POLY_SPLIT_BF16):
        say(f"dense prec {prec}")
        assert np.array_equal(bits(ph.eval_dense(basis, C, X, prec=prec)), bits(ph.eval_dense(basis, C, X, prec=prec)))
    gY = torch.from_numpy(W.rng_for(96).standard_normal((C.shape[0], X.shape[0]))).cuda()
    say("dense reverse mode")
    dC1, dX1 = ph.eval_dense_backward(basis, C, X, gY)
    dC2, dX2 = ph.eval_dense_backward(basis, C, X, gY)
    assert np.array_equal(bits(dC1), bits(dC2))
    assert torch.allclose(dX1, dX2, rtol=1e-13, atol=1e-13 * float(dX1.abs().max()))
    say("dense reverse mode, split")
    s1 = ph.eval_dense_backward(basis, C, X, gY, prec=ph.POLY_SPLIT_BF16)
    s2 = ph.eval_dense_backward(basis, C, X, gY, prec=ph.POLY_SPLIT_BF16)
    assert all(np.array_equal(bits(a), bits(b)) for a, b in zip(s1, s2))


def test_affine_paths_agree_to_rounding(ph):
    wl = W.sparse_quartic(seed=W.SEED_BASE + 97, n=12, npts=64)
    b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=12, max_exp=4)
    X = torch.from_numpy(wl.X * 0.35).cuda()
    D1, _ = ph.affine_normal(b, X, reg=1e-8)
    D2, _ = ph.affine_normal(b, X, reg=1e-8)
    assert torch.allclose(D1, D2, rtol=1e-12, atol=1e-12)
    Z = torch.from_numpy(W.rng_for(98).choice([-1.0, 1.0], size=(8, 12))).cuda()
    S1, _, h1 = ph.affine_normal_stochastic(b, X, Z, reg=1e-8, tol=1e-10, maxit=40)
    S2, _, h2 = ph.affine_normal_stochastic(b, X, Z, reg=1e-8, tol=1e-10, maxit=40)
    assert torch.allclose(S1, S2, rtol=1e-12, atol=1e-12)
    assert torch.equal(h1, h2)
