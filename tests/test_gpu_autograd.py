"""PolyEval (torch.autograd.Function over the library's reverse-mode kernel):
gradients w.r.t. coefficients and points against finite differences
(torch.autograd.gradcheck in FP64) and against the oracle's symbolic
derivatives."""
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


def test_gradcheck_small(ph):
    rng = W.rng_for(1201)
    n = 3
    polys = [W.random_poly(rng, n, 3, 6, integer=False), W.random_poly(rng, n, 4, 9, integer=False)]
    rp, E, C = W.csr_from_list(polys, n)
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=4)
    coefs = torch.from_numpy(C).cuda().requires_grad_(True)
    X = torch.from_numpy(W.points(1202, 5, n)).cuda().requires_grad_(True)
    say("gradcheck")
    assert torch.autograd.gradcheck(lambda c, x: ph.PolyEval.apply(c, x, b), (coefs, X), eps=1e-6, atol=1e-7,
                                    rtol=1e-6)


def test_backward_matches_symbolic(ph):
    rng = W.rng_for(1203)
    n = 6
    polys = [W.random_poly(rng, n, 4, 400, integer=False) for _ in range(3)]
    rp, E, C = W.csr_from_list(polys, n)
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=4)
    Xn = W.points(1204, 300, n)
    gYn = rng.standard_normal((3, 300))
    coefs = torch.from_numpy(C).cuda().requires_grad_(True)
    X = torch.from_numpy(Xn).cuda().requires_grad_(True)
    say("autograd backward")
    Y = ph.PolyEval.apply(coefs, X, b)
    Y.backward(torch.from_numpy(gYn).cuda())
    dXo, dCo = oracle.eval_backward(rp, E, C, Xn, gYn)
    aX, aC = oracle.eval_backward(rp, E, np.abs(C), np.abs(Xn), np.abs(gYn))
    assert (np.abs(X.grad.cpu().numpy() - dXo) <= 1e-12 * aX + 1e-300).all()
    assert (np.abs(coefs.grad.cpu().numpy() - dCo) <= 1e-12 * aC + 1e-300).all()
    # unit cotangent: dX is the sum of the gradients (symbolic jacobian of the oracle)
    X.grad = None
    Y = ph.PolyEval.apply(coefs.detach(), X, b)
    Y.sum().backward()
    G = oracle.grad_batch(rp, E, C, Xn)
    Ga = oracle.grad_batch(rp, E, np.abs(C), np.abs(Xn))
    assert (np.abs(X.grad.cpu().numpy() - G.sum(axis=0)) <= 1e-12 * Ga.sum(axis=0) + 1e-300).all()
