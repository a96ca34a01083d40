"""HIP path vs the CPU oracle, element by element, through the C ABI.

Integer work (exponent rows, term counts, order) is compared bit for bit;
coefficients of simplify/times are bit-exact too, because the merge sums every
run of equal monomials in the raw term order, the oracle's order.
Evaluation results are compared within |d| <= 1e-12 * sum_t |c_t v_t|
(FP64 rounding of a sum in a different order), and exactly at small integer
points with integer coefficients.
"""
import math
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


def dev_batch(ph, polys, n, max_exp=None):
    rp, E, C = W.csr_from_list(polys, n)
    return ph.batch_from_numpy(rp, E, C, n=n, max_exp=max_exp)


def assert_csr_bitwise(got, exp_rp, exp_E, exp_C):
    rp, E, C = got
    assert np.array_equal(rp, exp_rp), "row pointers differ"
    assert np.array_equal(E, exp_E), "exponent rows differ"
    assert C.view(np.uint64).tolist() == np.asarray(exp_C, dtype=np.float64).view(np.uint64).tolist(), \
        "coefficients differ bitwise"


def eval_tol(rp, E, C, X):
    """1e-12 * sum_t |c_t v_t| (condition-scaled bound)."""
    A = oracle.eval_batch(rp, E, np.abs(C), np.abs(X))
    return 1e-12 * A + 1e-300


def grad_tol(rp, E, C, X):
    """Per element: 1e-12 * sum_t |c_t e_j x^(e_t - u_j)|, the oracle's
    gradient of the polynomial with coefficients |c| at |x|."""
    return 1e-12 * oracle.grad_batch(rp, E, np.abs(C), np.abs(X)) + 1e-300


def hess_tol(rp, E, C, X):
    """Per element: 1e-12 * sum_t |d^2 (c_t x^e_t) / dx_j dx_k| at x."""
    return 1e-12 * oracle.hess_batch(rp, E, np.abs(C), np.abs(X)) + 1e-300


def backward_tol(rp, E, C, X, gY):
    """Per element of (dX, dC): 1e-12 times the same sums over absolute values
    (|gY|, |c|, |x|)."""
    aX, aC = oracle.eval_backward(rp, E, np.abs(C), np.abs(X), np.abs(gY))
    return 1e-12 * aX + 1e-300, 1e-12 * aC + 1e-300


# ------------------------------------------------------------------ simplify

def test_simplify_worked_examples(ph, golden):
    from conftest import poly_from_json
    g = golden["W5_mixed_simplify"]
    pe, pc = poly_from_json(g["p"], 4)
    qe, qc = poly_from_json(g["q"], 4)
    say("simplify W5")
    b = dev_batch(ph, [(np.vstack([pe, qe]), np.concatenate([pc, qc]))], 4)
    out = ph.batch_to_numpy(ph.simplify(b))
    xe, xc = poly_from_json(g["simplified"], 4)
    assert_csr_bitwise(out, np.array([0, xe.shape[0]]), xe, xc)
    g = golden["W1_scalar_workflow"]
    e, c = poly_from_json(g["input"], 3)
    say("simplify W1")
    out = ph.batch_to_numpy(ph.simplify(dev_batch(ph, [(e, c)], 3)))
    xe, xc = poly_from_json(g["simplified"], 3)
    assert_csr_bitwise(out, np.array([0, 4]), xe, xc)


@pytest.mark.parametrize("seed", range(6))
def test_simplify_random_batches(ph, seed):
    rng = W.rng_for(500 + seed)
    n = int(rng.integers(1, 9))
    d = int(rng.integers(1, 7))
    P = int(rng.integers(1, 40))
    polys = [W.random_poly(rng, n, d, int(rng.integers(0, 300)), integer=bool(seed % 2)) for _ in range(P)]
    tol = 0.0 if seed < 4 else 0.3
    rp, E, C = W.csr_from_list(polys, n)
    say(f"simplify random seed={seed} n={n} d={d} P={P} T={rp[-1]}")
    out = ph.batch_to_numpy(ph.simplify(ph.batch_from_numpy(rp, E, C, n=n, max_exp=d), tol))
    assert_csr_bitwise(out, *oracle.simplify_batch(rp, E, C, tol, n=n))


def test_simplify_batch_matrix_small(ph):
    """Polynomial-matrix batch with log-uniform entry sizes, including entries
    larger than one LDS tile (the key-range bisection path)."""
    wl = W.batch_matrix(seed=W.SEED_BASE + 30, entries=48, tmin=10, tmax=20000, npts=0)
    say(f"simplify matrix entries=48 T={wl.row_ptr[-1]} max entry={np.diff(wl.row_ptr).max()}")
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    out = ph.batch_to_numpy(ph.simplify(b))
    assert_csr_bitwise(out, *oracle.simplify_batch(wl.row_ptr, wl.exps, wl.coefs))


def test_simplify_giant_run(ph):
    """One monomial repeated far beyond a tile, plus a cancelling entry."""
    rng = W.rng_for(77)
    e = np.tile(np.array([[1, 2, 0]], np.uint8), (9000, 1))
    c = rng.standard_normal(9000)
    e2 = np.vstack([e[:5000], W.random_poly(rng, 3, 3, 3000)[0]])
    c2 = np.concatenate([c[:5000], rng.standard_normal(3000)])
    e3 = np.array([[1, 1, 1], [1, 1, 1]], np.uint8)
    c3 = np.array([2.5, -2.5])
    polys = [(e, c), (e2, c2), (e3, c3), (np.zeros((0, 3), np.uint8), np.zeros(0))]
    rp, E, C = W.csr_from_list(polys, 3)
    say("simplify giant run")
    out = ph.batch_to_numpy(ph.simplify(ph.batch_from_numpy(rp, E, C, n=3, max_exp=3)))
    assert_csr_bitwise(out, *oracle.simplify_batch(rp, E, C))
    assert out[0][3] - out[0][2] == 0    # cancelled entry is the structural zero


# ----------------------------------------------------------------------- mul

def test_mul_worked_examples(ph, golden):
    from conftest import poly_from_json
    g = golden["XY_square"]
    p = poly_from_json(g["p"], 2)
    say("mul (x+y)^2")
    out = ph.batch_to_numpy(ph.mul(dev_batch(ph, [p], 2), dev_batch(ph, [p], 2)))
    xe, xc = poly_from_json(g["square"], 2)
    assert_csr_bitwise(out, np.array([0, 3]), xe, xc)
    g = golden["W6_matrix_ops"]
    A = [poly_from_json(t, 2) for t in g["A"]]
    say("mul A.^2")
    ba = dev_batch(ph, A, 2, max_exp=1)
    out = ph.batch_to_numpy(ph.mul(ba, ba))
    exp = W.csr_from_list([oracle.mul(*a, *a, n=2) for a in A], 2)
    assert_csr_bitwise(out, *exp)
    assert out[0][3] - out[0][2] == 0


def test_mul_plain_small(ph):
    wl = W.plain_small()
    say("mul plain small (n=4, 200x200)")
    a = ph.batch_from_numpy([0, 200], wl.a_exps, wl.a_coefs, n=4, max_exp=6)
    b = ph.batch_from_numpy([0, 200], wl.b_exps, wl.b_coefs, n=4, max_exp=6)
    out = ph.batch_to_numpy(ph.mul(a, b))
    oe, oc = oracle.mul(wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs)
    assert_csr_bitwise(out, np.array([0, oe.shape[0]]), oe, oc)


@pytest.mark.parametrize("seed", range(6))
def test_mul_random_pairs(ph, seed):
    rng = W.rng_for(600 + seed)
    n = int(rng.integers(1, 7))
    d = int(rng.integers(1, 5))
    P = int(rng.integers(1, 12))
    A, B = [], []
    for _ in range(P):
        A.append(W.random_poly(rng, n, d, int(rng.integers(0, 120)), integer=bool(seed % 2)))
        B.append(W.random_poly(rng, n, d, int(rng.integers(0, 120)), integer=bool(seed % 2)))
    arp, aE, aC = W.csr_from_list(A, n)
    brp, bE, bC = W.csr_from_list(B, n)
    say(f"mul random seed={seed} n={n} P={P}")
    out = ph.batch_to_numpy(ph.mul(ph.batch_from_numpy(arp, aE, aC, n=n, max_exp=d),
                                   ph.batch_from_numpy(brp, bE, bC, n=n, max_exp=d)))
    assert_csr_bitwise(out, *oracle.mul_batch(arp, aE, aC, brp, bE, bC, n=n))


def test_mul_many_buckets(ph):
    """A pair with several hundred thousand raw terms (many key buckets),
    Gaussian coefficients: still bit-exact because runs are summed in (i, j)
    order."""
    wl = W.plain_large(seed=W.SEED_BASE + 40, terms=700, n=6, d=6)
    say("mul 700x700 n=6")
    a = ph.batch_from_numpy([0, 700], wl.a_exps, wl.a_coefs, n=6, max_exp=6)
    b = ph.batch_from_numpy([0, 700], wl.b_exps, wl.b_coefs, n=6, max_exp=6)
    out = ph.batch_to_numpy(ph.mul(a, b))
    oe, oc = oracle.mul(wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs)
    assert_csr_bitwise(out, np.array([0, oe.shape[0]]), oe, oc)


def test_mul_swapped_and_giant_run(ph):
    rng = W.rng_for(41)
    # |a| > |b| (rows become b's terms) with duplicates in a
    a = W.random_poly(rng, 3, 3, 900)
    b = W.random_poly(rng, 3, 3, 25)
    # a giant run: 3000 copies of x1 times 5 copies of x2 -> 15000 raw terms of x1*x2
    ga = (np.tile(np.array([[1, 0, 0]], np.uint8), (3000, 1)), rng.standard_normal(3000))
    gb = (np.tile(np.array([[0, 1, 0]], np.uint8), (5, 1)), rng.standard_normal(5))
    arp, aE, aC = W.csr_from_list([a, ga], 3)
    brp, bE, bC = W.csr_from_list([b, gb], 3)
    say("mul swapped + giant run")
    out = ph.batch_to_numpy(ph.mul(ph.batch_from_numpy(arp, aE, aC, n=3, max_exp=3),
                                   ph.batch_from_numpy(brp, bE, bC, n=3, max_exp=3)))
    rp, E, C = oracle.mul_batch(arp, aE, aC, brp, bE, bC, n=3)
    assert np.array_equal(out[0], rp) and np.array_equal(out[1], E)
    # pair 0 (integer coefficients) is bit-exact in any summation order
    assert np.array_equal(out[2][rp[0]:rp[1]], C[rp[0]:rp[1]])
    # pair 1 (one run of 15000 Gaussian products, summed in (i, j) order)
    assert out[2][rp[1]:rp[2]].view(np.uint64).tolist() == C[rp[1]:rp[2]].view(np.uint64).tolist()


def test_mul_errors(ph):
    a = dev_batch(ph, [(np.array([[200, 0]], np.uint8), np.array([1.0]))], 2, max_exp=200)
    with pytest.raises(ph.PolyError):
        ph.mul(a, a)            # 400 > 255 cannot be stored
    # 40 variables of 3-bit fields (120 bits) are no error: the product is
    # simplified over key words (times has no width limit in Section 3.3)
    wide = dev_batch(ph, [(np.ones((1, 40), np.uint8), np.array([1.5]))], 40, max_exp=3)
    rp, E, C = ph.batch_to_numpy(ph.mul(wide, wide))
    assert rp.tolist() == [0, 1] and (E == 2).all() and C.tolist() == [2.25]
    lie = dev_batch(ph, [(np.array([[5, 0]], np.uint8), np.array([1.0]))], 2, max_exp=2)
    with pytest.raises(ph.PolyError) as ei:
        ph.mul(lie, lie)        # exponent above the declared bound: device-detected
    assert ei.value.code == 5


# ------------------------------------------------------------------ jacobian

@pytest.mark.parametrize("seed", range(3))
def test_jacobian_bitwise(ph, seed):
    rng = W.rng_for(700 + seed)
    n = int(rng.integers(1, 12))
    polys = [W.random_poly(rng, n, 5, int(rng.integers(0, 700)), integer=False) for _ in range(int(rng.integers(1, 20)))]
    rp, E, C = W.csr_from_list(polys, n)
    say(f"jacobian seed={seed} n={n} P={len(polys)}")
    out = ph.batch_to_numpy(ph.jacobian(ph.batch_from_numpy(rp, E, C, n=n, max_exp=5)))
    assert_csr_bitwise(out, *oracle.jacobian_batch(rp, E, C, n=n))


# ---------------------------------------------------------------------- eval

@pytest.mark.parametrize("seed", range(3))
def test_eval_random(ph, seed):
    rng = W.rng_for(800 + seed)
    n = int(rng.integers(1, 20))
    polys = [W.random_poly(rng, n, 6, int(rng.integers(0, 3000)), integer=False) for _ in range(int(rng.integers(1, 9)))]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.points(801 + seed, int(rng.integers(1, 300)), n)
    say(f"eval seed={seed} n={n} P={len(polys)} N={X.shape[0]}")
    Y = ph.eval(ph.batch_from_numpy(rp, E, C, n=n, max_exp=6), torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = oracle.eval_batch(rp, E, C, X)
    assert (np.abs(Y - Yo) <= eval_tol(rp, E, C, X)).all()


def test_eval_integer_exact(ph):
    rng = W.rng_for(850)
    polys = [W.random_poly(rng, 4, 5, 50) for _ in range(5)] + [(np.zeros((0, 4), np.uint8), np.zeros(0))]
    rp, E, C = W.csr_from_list(polys, 4)
    X = W.integer_points(851, 70, 4, -2, 2)
    X[0] = 0.0                                       # 0^0 = 1
    say("eval integer exact")
    Y = ph.eval(ph.batch_from_numpy(rp, E, C, n=4, max_exp=5), torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.array_equal(Y, oracle.eval_batch(rp, E, C, X))
    assert (Y[-1] == 0).all()


def test_eval_wide_support_and_long_poly(ph):
    """Terms with more than eight variables (dense fallback) and one long
    polynomial split across the waves of a workgroup."""
    rng = W.rng_for(860)
    n = 12
    e = rng.integers(0, 3, size=(9000, n)).astype(np.uint8)
    c = rng.standard_normal(9000)
    rp = np.array([0, 9000], np.int64)
    X = W.points(861, 130, n)
    say("eval wide support")
    Y = ph.eval(ph.batch_from_numpy(rp, e, c, n=n, max_exp=2), torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = oracle.eval_batch(rp, e, c, X)
    assert (np.abs(Y - Yo) <= eval_tol(rp, e, c, X)).all()


def test_grad_hess(ph):
    rng = W.rng_for(870)
    n = 5
    polys = [W.random_poly(rng, n, 4, int(rng.integers(1, 400)), integer=False) for _ in range(4)]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.points(871, 100, n)
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=4)
    Xd = torch.from_numpy(X).cuda()
    say("grad")
    G = ph.grad(b, Xd, check=True).cpu().numpy()
    Go = oracle.grad_batch(rp, E, C, X)
    assert (np.abs(G - Go) <= grad_tol(rp, E, C, X)).all()
    say("hess")
    H = ph.hess(b, Xd, check=True).cpu().numpy()
    Ho = oracle.hess_batch(rp, E, C, X)
    assert (np.abs(H - Ho) <= hess_tol(rp, E, C, X)).all()
    assert np.array_equal(H, np.swapaxes(H, 2, 3))   # bitwise symmetric


def test_grad_hess_integer_exact(ph):
    rng = W.rng_for(880)
    n = 4
    polys = [W.random_poly(rng, n, 4, 60) for _ in range(3)]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.integer_points(881, 40, n)
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=4)
    Xd = torch.from_numpy(X).cuda()
    say("grad/hess integer")
    assert np.array_equal(ph.grad(b, Xd).cpu().numpy(), oracle.grad_batch(rp, E, C, X))
    assert np.array_equal(ph.hess(b, Xd).cpu().numpy(), oracle.hess_batch(rp, E, C, X))


def test_eval_backward(ph):
    rng = W.rng_for(890)
    n = 4
    polys = [W.random_poly(rng, n, 4, int(rng.integers(1, 300)), integer=False) for _ in range(3)]
    rp, E, C = W.csr_from_list(polys, n)
    X = W.points(891, 700, n)
    gY = rng.standard_normal((3, 700))
    say("eval backward")
    dX, dC = ph.eval_backward(ph.batch_from_numpy(rp, E, C, n=n, max_exp=4), torch.from_numpy(X).cuda(),
                              torch.from_numpy(gY).cuda(), check=True)
    dXo, dCo = oracle.eval_backward(rp, E, C, X, gY)
    tX, tC = backward_tol(rp, E, C, X, gY)
    assert (np.abs(dX.cpu().numpy() - dXo) <= tX).all()
    assert (np.abs(dC.cpu().numpy() - dCo) <= tC).all()


# --------------------------------------------------------------------- dense

@pytest.mark.parametrize("P,K,N", [(37, 300, 150), (130, 1000, 70)])
def test_dense_fp64(ph, P, K, N):
    wl = W.dense_shared(seed=900 + P, P=P, N=N, n=7, d=4, K=K)
    say(f"dense fp64 P={P} K={K} N={N}")
    Y = ph.eval_dense(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                      torch.from_numpy(wl.X).cuda(), prec=ph.POLY_FP64).cpu().numpy()
    Yo = oracle.eval_dense(wl.basis, wl.C, wl.X)
    A = oracle.eval_dense(wl.basis, np.abs(wl.C), np.abs(wl.X))
    assert (np.abs(Y - Yo) <= 1e-12 * A).all()


@pytest.mark.parametrize("S", [3, 4, 5])
def test_dense_split(ph, S):
    wl = W.dense_shared(seed=950, P=70, N=90, n=8, d=4, K=400)
    say(f"dense split S={S}")
    Y = ph.eval_dense(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                      torch.from_numpy(wl.X).cuda(), prec=ph.POLY_SPLIT_BF16, nslices=S).cpu().numpy()
    Yo = oracle.eval_dense(wl.basis, wl.C, wl.X)
    A = oracle.eval_dense(wl.basis, np.abs(wl.C), np.abs(wl.X))
    err = np.abs(Y - Yo) / A
    say(f"  S={S} max condition-scaled error {err.max():.3e}")
    # truncation after S digits, or the rounding floor of the shared FP32
    # group of diagonals >= 4 (about 2^-34 per 128-deep K-block)
    bound = max(2.0 ** -(8 * S - 12), 2.0 ** -33)
    assert err.max() <= bound
    if S >= 5:
        assert err.max() <= 1e-10


def test_dense_split_refuses_six_slices(ph):
    """A sixth digit would sit below the FP32 floor of the shared
    accumulator group of diagonals >= 4: refused on the host."""
    import ctypes
    size = ctypes.c_size_t()
    assert ph.lib().poly_eval_dense_workspace(8, 400, 70, 90, ph.POLY_SPLIT_BF16, 6, ctypes.byref(size)) == 1
    assert ph.lib().poly_eval_dense_workspace(8, 400, 70, 90, ph.POLY_SPLIT_BF16, 5, ctypes.byref(size)) == 0


def _dense_case(ph, wl, prec, S=5):
    Y = ph.eval_dense(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                      torch.from_numpy(wl.X).cuda(), prec=prec, nslices=S).cpu().numpy()
    Yo = oracle.eval_dense(wl.basis, wl.C, wl.X)
    A = oracle.eval_dense(wl.basis, np.abs(wl.C), np.abs(wl.X))
    return np.abs(Y - Yo) / A


def _block_scaled_reference(wl, kb=128):
    """sum over 128-deep K-blocks b of (sum_{k in b} |c_pk|) * max_{k in b} |v_k(x)|:
    the quantity the split path's truncation error is proportional to (its
    digits are relative to the largest monomial value of a block)."""
    V = oracle.eval_dense(wl.basis, np.eye(wl.basis.shape[0]), wl.X)    # [K, N] monomial values
    K = V.shape[0]
    ref = np.zeros((wl.C.shape[0], V.shape[1]))
    for k0 in range(0, K, kb):
        ref += np.abs(wl.C[:, k0:k0 + kb]).sum(1)[:, None] * np.abs(V[k0:k0 + kb]).max(0)[None, :]
    return ref


@pytest.mark.parametrize("split", [False, True])
def test_dense_high_degree(ph, split):
    """Degrees 0..14 in two variables: monomials of one factor word (<= 4),
    of up to three words (<= 12) and beyond the factor lists (exponent-row
    fallback) in the same K steps.  Monomial values span many binades inside
    a K-block, so the split result is held to its bound relative to the
    block-scaled reference."""
    wl = W.dense_shared(seed=960, P=45, N=77, n=2, d=14)
    say(f"dense high degree split={split}")
    prec = ph.POLY_SPLIT_BF16 if split else ph.POLY_FP64
    Y = ph.eval_dense(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                      torch.from_numpy(wl.X).cuda(), prec=prec, nslices=5).cpu().numpy()
    Yo = oracle.eval_dense(wl.basis, wl.C, wl.X)
    if split:
        err = np.abs(Y - Yo) / _block_scaled_reference(wl)
        assert err.max() <= max(2.0 ** -(8 * 5 - 12), 2.0 ** -33)
    else:
        A = oracle.eval_dense(wl.basis, np.abs(wl.C), np.abs(wl.X))
        assert (np.abs(Y - Yo) <= 1e-12 * A).all()


@pytest.mark.parametrize("split", [False, True])
def test_dense_several_workgroup_tiles(ph, split):
    """P = 300 (two row workgroups of the split tile, a partial 32-row block),
    K = 700 (six 128-deep K-blocks, ragged last step), N = 130 (ragged
    point tile)."""
    wl = W.dense_shared(seed=961, P=300, N=130, n=9, d=4, K=700)
    say(f"dense tiles split={split}")
    err = _dense_case(ph, wl, ph.POLY_SPLIT_BF16 if split else ph.POLY_FP64)
    assert err.max() <= (1e-10 if split else 1e-12)


@pytest.mark.parametrize("rows", [64, 128])
def test_dense_fp64_row_tiles(ph, rows):
    """The FP64 contraction and the reverse mode's dC with 64 or 128 rows per
    workgroup (the dense_f64_rows tunable), and dX beside them: P = 300
    leaves a partial row tile either way, K = 700 a ragged last step, N = 130
    a ragged point tile; degrees to 14 in two variables take every
    factor-list form."""
    old = ph.tune_get("dense_f64_rows")
    try:
        ph.tune_set("dense_f64_rows", rows)
        for wl in (W.dense_shared(seed=962, P=300, N=130, n=9, d=4, K=700), W.dense_shared(seed=963, P=45, N=77, n=2, d=14)):
            say(f"dense fp64 rows={rows} P={wl.C.shape[0]} K={wl.basis.shape[0]}")
            assert _dense_case(ph, wl, ph.POLY_FP64).max() <= 1e-12
            # the reverse mode's dC takes the same row tile
            P, Kr = wl.C.shape
            gY = W.rng_for(964).standard_normal((P, wl.X.shape[0]))
            dC, dX = ph.eval_dense_backward(torch.from_numpy(wl.basis).cuda(), torch.from_numpy(wl.C).cuda(),
                                            torch.from_numpy(wl.X).cuda(), torch.from_numpy(gY).cuda())
            rp = np.arange(P + 1, dtype=np.int64) * Kr
            E = np.tile(wl.basis, (P, 1))
            dXo, dCo = oracle.eval_backward(rp, E, wl.C.ravel(), wl.X, gY)
            aX, aC = oracle.eval_backward(rp, E, np.abs(wl.C.ravel()), np.abs(wl.X), np.abs(gY))
            assert (np.abs(dC.cpu().numpy().ravel() - dCo) <= 1e-12 * aC + 1e-300).all()
            assert (np.abs(dX.cpu().numpy() - dXo) <= 1e-12 * aX + 1e-300).all()
    finally:
        ph.tune_set("dense_f64_rows", old)


def test_dense_empty_basis(ph):
    """K = 0: every output is the empty sum, 0."""
    basis = torch.zeros((0, 3), dtype=torch.uint8, device="cuda")
    C = torch.zeros((5, 0), dtype=torch.float64, device="cuda")
    X = torch.rand((9, 3), dtype=torch.float64, device="cuda")
    for prec in (ph.POLY_FP64, ph.POLY_SPLIT_BF16):
        Y = ph.eval_dense(basis, C, X, prec=prec).cpu().numpy()
        assert Y.shape == (5, 9) and not Y.any()
