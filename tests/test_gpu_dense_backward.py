"""Reverse mode of the shared-monomial-set contraction on FP64 MFMA
(poly_eval_dense_backward) against the oracle's reverse mode of eval on the
same batch stored as CSR, element by element within 1e-12 times the same
sums over |gY|, |c|, |x|; point and monomial counts that leave ragged
tiles, degrees past the factor lists, and autograd (gradcheck) through
PolyEvalDense."""
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


def as_csr(basis, C):
    P, K = C.shape
    return np.arange(P + 1, dtype=np.int64) * K, np.tile(basis, (P, 1)), C.ravel()


@pytest.mark.parametrize("P,K,N,n,d", [(37, 300, 150, 7, 4), (70, 130, 257, 5, 4), (9, 56, 40, 2, 14)])
def test_dense_backward_matches_oracle(ph, P, K, N, n, d):
    wl = W.dense_shared(seed=4000 + P, P=P, N=N, n=n, d=d, K=K)
    Kr = wl.basis.shape[0]
    gY = W.rng_for(4001 + P).standard_normal((P, N))
    say(f"dense backward P={P} K={Kr} N={N} n={n} d={d}")
    dC, dX = ph.eval_dense_backward(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                                    torch.from_numpy(wl.X).cuda(), torch.from_numpy(gY).cuda())
    rp, E, Cf = as_csr(wl.basis, wl.C)
    dXo, dCo = oracle.eval_backward(rp, E, Cf, wl.X, gY)
    aX, aC = oracle.eval_backward(rp, E, np.abs(Cf), np.abs(wl.X), np.abs(gY))
    assert (np.abs(dC.cpu().numpy().ravel() - dCo) <= 1e-12 * aC + 1e-300).all()
    assert (np.abs(dX.cpu().numpy() - dXo) <= 1e-12 * aX + 1e-300).all()


def test_dense_backward_gradcheck(ph):
    wl = W.dense_shared(seed=4010, P=5, N=6, n=3, d=3, K=20)
    basis = torch.from_numpy(wl.basis).cuda()
    C = torch.from_numpy(wl.C).cuda().requires_grad_(True)
    X = torch.from_numpy(wl.X).cuda().requires_grad_(True)
    say("dense gradcheck")
    assert torch.autograd.gradcheck(lambda c, x: ph.PolyEvalDense.apply(c, x, basis), (C, X), eps=1e-6, atol=1e-7,
                                    rtol=1e-6)
