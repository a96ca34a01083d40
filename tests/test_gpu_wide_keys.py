"""Keys wider than 64 bits: simplify, times and mtimes of polynomials whose
exponents do not fit one 64-bit word (n * bit_width(max_exp) > 64), and
batches whose (polynomial, monomial) composite key does not (many entries in
20 variables, as in the 4,096-entry polynomial matrix), through the
device-wide sort over key words.  Every result is compared bit for bit with the oracle, which orders
exponent rows lexicographically and has no key width at all; the composite
case is also compared with the one-workgroup-per-polynomial path."""
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
    old = ph.tune_get("simplify_wide_min")
    yield ph
    ph.tune_set("simplify_wide_min", old)


def _same(ph, got, want):
    grp, gE, gC = ph.batch_to_numpy(got)
    rp, E, C = want
    assert np.array_equal(grp, rp), "row pointers differ"
    assert np.array_equal(gE, E), "exponent rows differ"
    assert np.array_equal(gC.view(np.uint64), np.asarray(C, np.float64).view(np.uint64)), "coefficients differ"


def _dup_batch(seed, P, n, d, tmin, tmax, integer=False):
    """P entries of terms drawn with replacement (repeated monomials to
    merge), sizes log-uniform in [tmin, tmax]."""
    rng = W.rng_for(seed)
    polys = []
    for _ in range(P):
        t = int(np.exp(rng.uniform(np.log(tmin), np.log(tmax))))
        polys.append(W.random_poly(rng, n, d, t, integer=integer))
    return W.csr_from_list(polys, n)


@pytest.mark.parametrize("n,d,P", [(30, 7, 40), (100, 7, 12), (255, 3, 6)])
def test_simplify_exponents_past_64_bits(ph, n, d, P):
    """n * bit_width(d) = 90, 300, 510 bits: 2, 5 and 9 key words."""
    rp, E, C = _dup_batch(7000 + n, P, n, d, 5, 3000)
    # exponents reach d so the declared bound is exercised at its edge
    E[::7, n // 2] = d
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=d)
    say(f"simplify n={n} max_exp={d}: {P} entries, {b.nterms} terms")
    _same(ph, ph.simplify(b), oracle.simplify_batch(rp, E, C, n=n))


def test_simplify_composite_past_64_bits(ph):
    """n = 20, max_exp 6 (60 bits of fields) but 300 entries: the composite
    key needs 9 + 57 bits; the word path and the per-entry path agree bit for
    bit and with the oracle."""
    rp, E, C = _dup_batch(7100, 300, 20, 6, 10, 9000)
    b = ph.batch_from_numpy(rp, E, C, n=20, max_exp=6)
    say(f"simplify composite: 300 entries, {b.nterms} terms")
    want = oracle.simplify_batch(rp, E, C, n=20)
    ph.tune_set("simplify_wide_min", 1)
    _same(ph, ph.simplify(b), want)
    ph.tune_set("simplify_wide_min", 1 << 62)
    _same(ph, ph.simplify(b), want)


def test_simplify_words_empty_entries_and_total_cancellation(ph):
    """Empty entries between full ones, and an entry whose terms all cancel,
    on the word path (30 variables of 3-bit fields)."""
    n = 30
    rng = W.rng_for(7250)
    E1, C1 = W.random_poly(rng, n, 5, 300, integer=False)
    E2, C2 = W.random_poly(rng, n, 5, 200, integer=False)
    empty = (np.zeros((0, n), np.uint8), np.zeros(0))
    polys = [empty, (E1, C1), empty, empty, (np.vstack([E2, E2]), np.concatenate([C2, -C2])), (E2, C2), empty]
    rp, E, C = W.csr_from_list(polys, n)
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=7)
    say("simplify words: empty entries, a fully cancelled entry")
    _same(ph, ph.simplify(b), oracle.simplify_batch(rp, E, C, n=n))


def test_simplify_words_drop_zeros_and_tolerance(ph):
    """Exact cancellation and a tolerance on the word path."""
    n = 40
    rng = W.rng_for(7200)
    E1, C1 = W.random_poly(rng, n, 4, 500, integer=False)
    E = np.vstack([E1, E1, E1[:100]])
    C = np.concatenate([C1, -C1, 1e-12 * np.ones(100)])
    rp = np.array([0, E.shape[0]], np.int64)
    b = ph.batch_from_numpy(rp, E, C, n=n, max_exp=4)
    say("simplify words: cancellation and tolerance")
    _same(ph, ph.simplify(b), oracle.simplify_batch(rp, E, C, n=n))
    _same(ph, ph.simplify(b, tol=1e-9), oracle.simplify_batch(rp, E, C, tol=1e-9, n=n))


def test_simplify_words_exponent_bound(ph):
    """An exponent above the declared bound, found on the device."""
    rp, E, C = _dup_batch(7300, 4, 30, 5, 10, 50)
    E[3, 7] = 6
    b = ph.batch_from_numpy(rp, E, C, n=30, max_exp=5)
    say("simplify words: exponent above max_exp")
    with pytest.raises(ph.PolyError) as ex:
        ph.simplify(b)
    assert ex.value.code == 5


@pytest.mark.parametrize("n,P,ta,tb", [(30, 6, 60, 80), (36, 1, 2000, 1500)])
def test_mul_exponents_past_64_bits(ph, n, P, ta, tb):
    """times with n * bit_width(4 + 4) = 120 or 144 bits: the raw products
    are written as rows in the order of the definition and simplified over
    key words; one pair of 3M raw terms spans many merge tiles."""
    rng = W.rng_for(7400 + n)
    A = [W.random_poly(rng, n, 4, ta, integer=False) for _ in range(P)]
    B = [W.random_poly(rng, n, 4, tb, integer=False) for _ in range(P)]
    ra, rb = W.csr_from_list(A, n), W.csr_from_list(B, n)
    a = ph.batch_from_numpy(*ra, n=n, max_exp=4)
    b = ph.batch_from_numpy(*rb, n=n, max_exp=4)
    say(f"mul n={n}: {P} pairs, {sum(x[0].shape[0] * y[0].shape[0] for x, y in zip(A, B))} raw terms")
    _same(ph, ph.mul(a, b), oracle.mul_batch(*ra, *rb, n=n))


def test_mtimes_exponents_past_64_bits(ph):
    n = 24
    rng = W.rng_for(7500)
    A = [W.random_poly(rng, n, 4, 40, integer=False) for _ in range(4)]
    B = [W.random_poly(rng, n, 4, 30, integer=False) for _ in range(6)]
    ra, rb = W.csr_from_list(A, n), W.csr_from_list(B, n)
    a = ph.batch_from_numpy(*ra, n=n, max_exp=4)
    b = ph.batch_from_numpy(*rb, n=n, max_exp=4)
    say("mtimes n=24, 2x2 by 2x3")
    _same(ph, ph.mtimes(a, b, 2, 2, 3), oracle.mtimes(*ra, *rb, 2, 2, 3, n=n))
