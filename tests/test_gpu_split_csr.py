"""prec = POLY_SPLIT_BF16 on the sparse entry points (poly_eval, poly_grad,
poly_hess, poly_eval_backward) for a CSR batch that is one shared monomial
set.

Values, gradients and Hessians from the split contraction are held to the
oracle's symbolic derivatives: per element within the split scheme's bound,
max(2^-(8S-12), 2^-33) times the block-scaled reference
sum_blocks (sum_{k in block} |c'_k|) * max_{k in block} |v'_k(x)| of the
contraction actually performed (c', v' the derived coefficients and
monomials), and within 1e-10 of the condition number sum |c v| (R20's gate)
where the monomial values of a block share a binade.  Hessians are
bitwise symmetric.  A batch whose polynomials have different lengths is
refused by the host; one with equal lengths but different rows is reported
by the device status."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
S = 5


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


def shared_batch(P, n, d, K, seed):
    rng = W.rng_for(seed)
    B = W.basis(n, d)
    B = B[rng.permutation(B.shape[0])[:K]]
    C = rng.standard_normal((P, B.shape[0]))
    rp = np.arange(P + 1, dtype=np.int64) * B.shape[0]
    return B, C, rp, np.tile(B, (P, 1)), C.ravel()


def block_ref(Bd, Cd, X, kb=128):
    """sum over K-blocks of (sum |c'|) * max |v'| for coefficients Cd [P, K]
    over monomials Bd [K, n]."""
    V = oracle.eval_dense(Bd, np.eye(Bd.shape[0]), X)
    ref = np.zeros((Cd.shape[0], X.shape[0]))
    for k0 in range(0, Bd.shape[0], kb):
        ref += np.abs(Cd[:, k0:k0 + kb]).sum(1)[:, None] * np.abs(V[k0:k0 + kb]).max(0)[None, :]
    return ref


def derived(B, C, j, k=None):
    """The derivative's contraction: rows e - u_j (- u_k), coefficients m c."""
    ej = B[:, j].astype(np.int64)
    if k is None:
        m = ej
    else:
        m = ej * (B[:, k].astype(np.int64) - (1 if k == j else 0))
    Bd = B.astype(np.int64).copy()
    keep = m > 0
    Bd[keep, j] -= 1
    if k is not None:
        Bd[keep, k] -= 1
    return Bd.astype(np.uint8), C * m[None, :]


BOUND = max(2.0 ** -(8 * S - 12), 2.0 ** -33)


def test_eval_split_csr(ph):
    B, C, rp, E, Cf = shared_batch(P=37, n=6, d=4, K=210, seed=3100)
    X = W.points(3101, 150, 6)
    b = ph.batch_from_numpy(rp, E, Cf, n=6, max_exp=4)
    say("eval split, shared set of 210 monomials, 37 polynomials, 150 points")
    Y = ph.eval(b, torch.from_numpy(X).cuda(), check=True, prec=ph.POLY_SPLIT_BF16, nslices=S).cpu().numpy()
    Yo = oracle.eval_batch(rp, E, Cf, X)
    A = oracle.eval_batch(rp, E, np.abs(Cf), np.abs(X))
    assert (np.abs(Y - Yo) <= BOUND * block_ref(B, C, X)).all()
    assert (np.abs(Y - Yo) <= 1e-10 * A).all()


def test_grad_split_csr(ph):
    n = 5
    B, C, rp, E, Cf = shared_batch(P=20, n=n, d=4, K=126, seed=3110)
    X = W.points(3111, 90, n)
    b = ph.batch_from_numpy(rp, E, Cf, n=n, max_exp=4)
    say("grad split, shared set of 126 monomials, 20 polynomials, 90 points")
    G = ph.grad(b, torch.from_numpy(X).cuda(), check=True, prec=ph.POLY_SPLIT_BF16, nslices=S).cpu().numpy()
    Go = oracle.grad_batch(rp, E, Cf, X)
    for j in range(n):
        Bd, Cd = derived(B, C, j)
        assert (np.abs(G[:, :, j] - Go[:, :, j]) <= BOUND * block_ref(Bd, Cd, X) + 1e-300).all()


def test_hess_split_csr(ph):
    n = 4
    B, C, rp, E, Cf = shared_batch(P=9, n=n, d=4, K=70, seed=3120)
    X = W.points(3121, 70, n)
    b = ph.batch_from_numpy(rp, E, Cf, n=n, max_exp=4)
    say("hess split, shared set of 70 monomials, 9 polynomials, 70 points")
    H = ph.hess(b, torch.from_numpy(X).cuda(), check=True, prec=ph.POLY_SPLIT_BF16, nslices=S).cpu().numpy()
    Ho = oracle.hess_batch(rp, E, Cf, X)
    assert np.array_equal(H, np.swapaxes(H, 2, 3))
    for j in range(n):
        for k in range(j, n):
            Bd, Cd = derived(B, C, j, k)
            assert (np.abs(H[:, :, j, k] - Ho[:, :, j, k]) <= BOUND * block_ref(Bd, Cd, X) + 1e-300).all()


def test_split_csr_requires_a_shared_set(ph):
    B, C, rp, E, Cf = shared_batch(P=6, n=4, d=3, K=30, seed=3130)
    X = torch.from_numpy(W.points(3131, 20, 4)).cuda()
    E2 = E.copy()
    E2[35] = E2[36]   # polynomial 1 lists another row in slot 5
    b = ph.batch_from_numpy(rp, E2, Cf, n=4, max_exp=3)
    say("split on unequal rows: device status")
    with pytest.raises(ph.PolyError) as ex:
        ph.eval(b, X, check=True, prec=ph.POLY_SPLIT_BF16, nslices=S)
    assert ex.value.code == 6
    rp2 = np.array([0, 30, 59, 90], np.int64)   # unequal lengths: refused on the host
    b2 = ph.batch_from_numpy(rp2, E[:90], Cf[:90], n=4, max_exp=3)
    with pytest.raises(ph.PolyError) as ex:
        ph.grad(b2, X, prec=ph.POLY_SPLIT_BF16, nslices=S)
    assert ex.value.code == 6
    say("split reverse mode on unequal rows and lengths")
    gY = torch.ones((6, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(ph.PolyError) as ex:
        ph.eval_backward(b, X, gY, check=True, prec=ph.POLY_SPLIT_BF16, nslices=S)
    assert ex.value.code == 6
    with pytest.raises(ph.PolyError) as ex:
        ph.eval_backward(b2, X, gY[:3], prec=ph.POLY_SPLIT_BF16, nslices=S)
    assert ex.value.code == 6


def test_eval_backward_split_csr(ph):
    """Reverse mode with prec = POLY_SPLIT_BF16: dC per term (the P x K
    matrix in CSR order) and dX on the split scheme against the oracle,
    within the bound relative to the block-scaled references and within
    1e-10 of the sums over absolute values."""
    from conftest import block_scaled_reference, monomial_values, split_dx_reference
    n = 6
    B, C, rp, E, Cf = shared_batch(P=45, n=n, d=4, K=190, seed=3140)
    X = W.points(3141, 300, n)
    gY = W.rng_for(3142).standard_normal((45, 300))
    b = ph.batch_from_numpy(rp, E, Cf, n=n, max_exp=4)
    say("eval_backward split, shared set of 190 monomials, 45 polynomials, 300 points")
    dX, dC = ph.eval_backward(b, torch.from_numpy(X).cuda(), torch.from_numpy(gY).cuda(), check=True,
                              prec=ph.POLY_SPLIT_BF16, nslices=S)
    dXo, dCo = oracle.eval_backward(rp, E, Cf, X, gY)
    aX, aC = oracle.eval_backward(rp, E, np.abs(Cf), np.abs(X), np.abs(gY))
    err = np.abs(dC.cpu().numpy() - dCo).reshape(45, -1)
    assert (err <= BOUND * block_scaled_reference(monomial_values(B, X), gY) + 1e-300).all()
    assert (err <= 1e-10 * aC.reshape(45, -1) + 1e-300).all()
    errx = np.abs(dX.cpu().numpy() - dXo)
    assert (errx <= BOUND * split_dx_reference(B, C, X, gY) + 1e-12 * aX + 1e-300).all()
    assert (errx <= 1e-10 * aX + 1e-300).all()
