"""Reverse mode of the shared-monomial-set contraction
(poly_eval_dense_backward) against the oracle's reverse mode of eval on the
same batch stored as CSR.  FP64: element by element within 1e-12 times the
same sums over |gY|, |c|, |x|.  Split dC (3 to 5 BF16 digits): within the
truncation bound relative to the block-scaled reference, and at 5 digits
within 1e-10 of sum_pt |gY v_k|.  Point and monomial counts that leave
ragged tiles, degrees past the factor lists, degenerate sizes, refused
limits, and autograd (gradcheck) through PolyEvalDense."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from conftest import block_scaled_reference, monomial_values, split_dx_reference

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


SPLIT_CASES = [(300, 130, 300, 7, 4), (37, 300, 150, 7, 4), (9, 56, 40, 2, 14), (20, 200, 100, 40, 2),
               (33, 70, 5, 4, 3), (40, 50, 4500, 3, 4)]


@pytest.mark.parametrize("S", [3, 4, 5])
@pytest.mark.parametrize("P,K,N,n,d", SPLIT_CASES)
def test_dense_backward_split(ph, S, P, K, N, n, d):
    """dC = gY V^T and dX through W = C^T gY on BF16 digits against the
    oracle's reverse mode: P = 300 spans two row workgroups and a partial
    32-row block (and three 128-polynomial blocks of W), K = 130 three
    monomial tiles with a ragged one, N = 300 three 128-point blocks with a
    ragged 32-point step; degrees to 14 take the factor lists' longer forms
    and the exponent-row fallback; n = 40 stages more coordinates per thread;
    N = 5 is one partial step; N = 4,500 two chunks of W.  Errors are held to the truncation bound
    relative to the block-scaled references (plus 1e-12 of the FP64 sums for
    dX's FP64 contraction with the derivatives), and at 5 digits to 1e-10 of
    the condition sums over absolute values."""
    wl = W.dense_shared(seed=4100 + P + N, P=P, N=N, n=n, d=d, K=K)
    Kr = wl.basis.shape[0]
    gY = W.rng_for(4101 + P + N).standard_normal((P, N))
    say(f"dense backward split S={S} P={P} K={Kr} N={N} n={n} d={d}")
    args = [torch.from_numpy(a).cuda() for a in (wl.basis, wl.C, wl.X, gY)]
    dC, dX = ph.eval_dense_backward(*args, prec=ph.POLY_SPLIT_BF16, nslices=S)
    rp, E, Cf = as_csr(wl.basis, wl.C)
    dXo, dCo = oracle.eval_backward(rp, E, Cf, wl.X, gY)
    aX, aC = oracle.eval_backward(rp, E, np.abs(Cf), np.abs(wl.X), np.abs(gY))
    bound = max(2.0 ** -(8 * S - 12), 2.0 ** -33)
    err = np.abs(dC.cpu().numpy() - dCo.reshape(P, Kr))
    ref = block_scaled_reference(monomial_values(wl.basis, wl.X), gY)
    say(f"  dC max block-scaled error {(err / ref).max():.3e}")
    assert (err <= bound * ref + 1e-300).all()
    errx = np.abs(dX.cpu().numpy() - dXo)
    refx = split_dx_reference(wl.basis, wl.C, wl.X, gY)
    say(f"  dX max block-scaled error {(errx / (refx + 1e-300)).max():.3e}")
    assert (errx <= bound * refx + 1e-12 * aX + 1e-300).all()
    if S == 5:
        assert (err <= 1e-10 * aC.reshape(P, Kr) + 1e-300).all()
        assert (errx <= 1e-10 * aX + 1e-300).all()


def test_dense_backward_split_degenerate(ph):
    """No points (dC is the empty sum, 0), no monomials, no polynomials, and a
    zero cotangent (every scale at its floor: dC exactly 0)."""
    wl = W.dense_shared(seed=4130, P=6, N=40, n=3, d=3, K=15)
    basis, C, X = (torch.from_numpy(a).cuda() for a in (wl.basis, wl.C, wl.X))
    split = dict(prec=ph.POLY_SPLIT_BF16, nslices=4)
    say("split dC: N = 0")
    dC, dX = ph.eval_dense_backward(basis, C, X[:0], torch.zeros((6, 0), dtype=torch.float64, device="cuda"), **split)
    assert dC.shape == (6, 15) and not dC.any() and dX.shape == (0, 3)
    say("split dC: K = 0")
    dC, dX = ph.eval_dense_backward(basis[:0], C[:, :0].contiguous(), X, torch.ones((6, 40), dtype=torch.float64,
                                                                                  device="cuda"), **split)
    assert dC.shape == (6, 0) and not dX.any()
    say("split dC: P = 0")
    dC, dX = ph.eval_dense_backward(basis, C[:0], X, torch.zeros((0, 40), dtype=torch.float64, device="cuda"), **split)
    assert dC.shape == (0, 15) and not dX.any()
    say("split dC: zero cotangent")
    dC, _ = ph.eval_dense_backward(basis, C, X, torch.zeros((6, 40), dtype=torch.float64, device="cuda"), **split)
    assert not dC.any()


def test_dense_backward_split_limits(ph):
    """Digit counts outside 3..5 and n past the staged coordinates are
    refused before any launch."""
    wl = W.dense_shared(seed=4140, P=3, N=4, n=65, d=1)
    args = [torch.from_numpy(a).cuda() for a in (wl.basis, wl.C, wl.X)]
    gY = torch.ones((3, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ph.PolyError) as ex:
        ph.eval_dense_backward(*args, gY, want_dX=False, prec=ph.POLY_SPLIT_BF16, nslices=6)
    assert ex.value.code == 1
    with pytest.raises(ph.PolyError) as ex:
        ph.eval_dense_backward(*args, gY, want_dX=False, prec=ph.POLY_SPLIT_BF16, nslices=5)
    assert ex.value.code == 6


def test_dense_autograd_split_backward(ph):
    """PolyEvalDense with prec=POLY_SPLIT_BF16 takes the split dC and dX of
    eval_dense_backward, bit for bit."""
    wl = W.dense_shared(seed=4150, P=40, N=90, n=5, d=4, K=100)
    basis = torch.from_numpy(wl.basis).cuda()
    C = torch.from_numpy(wl.C).cuda().requires_grad_(True)
    X = torch.from_numpy(wl.X).cuda().requires_grad_(True)
    gY = torch.from_numpy(W.rng_for(4151).standard_normal((40, 90))).cuda()
    say("dense autograd, split")
    ph.PolyEvalDense.apply(C, X, basis, ph.POLY_SPLIT_BF16, 5).backward(gY)
    dC, dX = ph.eval_dense_backward(basis, C.detach(), X.detach(), gY, prec=ph.POLY_SPLIT_BF16, nslices=5)
    assert torch.equal(C.grad, dC) and torch.equal(X.grad, dX)
