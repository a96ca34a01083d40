"""Products of polynomial matrices (Section 3.3, mtimes) through the C-ABI,
bit-exact against the oracle: the raw products of A_ik and B_kj
concatenated over k, then simplify."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def _batch(ph, polys, n, max_exp):
    rp, E, C = W.csr_from_list(polys, n)
    return ph.batch_from_numpy(rp, E, C, n=n, max_exp=max_exp), (rp, E, C)


def _same(ph, got, want):
    grp, gE, gC = ph.batch_to_numpy(got)
    rp, E, C = want
    assert np.array_equal(grp, rp), "row pointers differ"
    assert np.array_equal(gE, E), "exponent rows differ"
    assert gC.view(np.uint64).tolist() == np.asarray(C, np.float64).view(np.uint64).tolist(), "coefficients differ"


def _case(ph, A, B, I, K, J, n, d, tol=0.0):
    a, ra = _batch(ph, A, n, d)
    b, rb = _batch(ph, B, n, d)
    got = ph.mtimes(a, b, I, K, J, tol=tol)
    _same(ph, got, oracle.mtimes(*ra, *rb, I, K, J, tol=tol, n=n))
    return got


def test_paper_matrix_square(ph):
    g = json.load(open(os.path.join(HERE, "golden", "worked_examples.json")))["W6_matrix_ops"]
    n = g["n"]
    A = [(np.array([t[1] for t in e], np.uint8).reshape(-1, n), np.array([t[0] for t in e], float)) for e in g["A"]]
    say("mtimes: A^2 of Section 3.3")
    _case(ph, A, A, 2, 2, 2, n, 1)


@pytest.mark.parametrize("I,K,J", [(3, 4, 2), (1, 5, 1), (4, 1, 3), (2, 2, 2)])
def test_random_shapes(ph, I, K, J):
    """Gaussian coefficients (so only the defined summation order matches),
    repeated and cancelling terms, some zero entries."""
    rng = W.rng_for(3500 + 100 * I + 10 * K + J)
    n, d = 3, 3
    A = [W.random_poly(rng, n, d, int(rng.integers(0, 15)), integer=False) for _ in range(I * K)]
    B = [W.random_poly(rng, n, d, int(rng.integers(0, 15)), integer=False) for _ in range(K * J)]
    say(f"mtimes: {I}x{K} by {K}x{J}")
    _case(ph, A, B, I, K, J, n, d)


def test_several_tiles(ph):
    """8 x 8 matrices of 40-term entries: 12,800 raw terms per output entry."""
    rng = W.rng_for(3601)
    n, d = 5, 4
    A = [W.random_poly(rng, n, d, 40, integer=False) for _ in range(64)]
    B = [W.random_poly(rng, n, d, 40, integer=False) for _ in range(64)]
    say("mtimes: 8x8 by 8x8, 40 terms per entry")
    _case(ph, A, B, 8, 8, 8, n, d)


def test_tolerance_and_mpower(ph):
    rng = W.rng_for(3602)
    n, d = 2, 2
    A = [W.random_poly(rng, n, d, 4) for _ in range(9)]
    a, ra = _batch(ph, A, n, d)
    say("mpower: A^3, 3x3")
    got = ph.mpower(a, 3, 3)
    want = oracle.mtimes(*ra, *oracle.mtimes(*ra, *ra, 3, 3, 3, n=n), 3, 3, 3, n=n)
    _same(ph, got, want)
    _case(ph, A, A, 3, 3, 3, n, d, tol=50.0)


def test_empty(ph):
    n = 2
    a, _ = _batch(ph, [], n, 1)
    b, _ = _batch(ph, [(np.array([[1, 0]], np.uint8), np.array([2.0]))] * 3, n, 1)
    got = ph.mtimes(a, b, 0, 1, 3)
    assert got.npolys == 0


def test_paper_sum_and_prod(ph):
    """Section 3.3: sum(A, 1) = [x1, 1 + x2], prod(A, 2) = [x1; 0]."""
    g = json.load(open(os.path.join(HERE, "golden", "worked_examples.json")))["W6_matrix_ops"]
    n = g["n"]
    A = [(np.array([t[1] for t in e], np.uint8).reshape(-1, n), np.array([t[0] for t in e], float)) for e in g["A"]]
    a, ra = _batch(ph, A, n, 1)
    say("msum / mprod: Section 3.3 example")
    _same(ph, ph.msum(a, 2, 2, 1), oracle.msum(*ra, 2, 2, 1, n=n))
    _same(ph, ph.mprod(a, 2, 2, 2), oracle.mprod(*ra, 2, 2, 2, n=n))


@pytest.mark.parametrize("dim", [1, 2])
def test_sum_and_prod_random(ph, dim):
    """3 x 4 matrices of unsimplified entries with Gaussian coefficients (the
    summation order matters), some zero entries, with and without tol."""
    rng = W.rng_for(3700 + dim)
    n, d, R, C = 3, 2, 3, 4
    A = [W.random_poly(rng, n, d, int(rng.integers(0, 25)), integer=False) for _ in range(R * C)]
    a, ra = _batch(ph, A, n, d)
    for tol in (0.0, 0.5):
        say(f"msum / mprod: 3x4 along dim {dim}, tol {tol}")
        _same(ph, ph.msum(a, R, C, dim, tol=tol), oracle.msum(*ra, R, C, dim, tol=tol, n=n))
        _same(ph, ph.mprod(a, R, C, dim, tol=tol), oracle.mprod(*ra, R, C, dim, tol=tol, n=n))


def test_sum_and_prod_degenerate(ph):
    """An empty dimension (structural zeros / constant 1) and a dimension of
    length one (the simplified entries)."""
    n = 2
    a, ra = _batch(ph, [], n, 1)
    say("msum / mprod: empty dimension")
    _same(ph, ph.msum(a, 3, 0, 2), oracle.msum(*ra, 3, 0, 2, n=n))
    _same(ph, ph.mprod(a, 3, 0, 2), oracle.mprod(*ra, 3, 0, 2, n=n))
    rng = W.rng_for(3710)
    A = [W.random_poly(rng, n, 3, 8, integer=False) for _ in range(3)]
    a, ra = _batch(ph, A, n, 3)
    say("msum / mprod: one column")
    _same(ph, ph.msum(a, 3, 1, 2), oracle.msum(*ra, 3, 1, 2, n=n))
    _same(ph, ph.mprod(a, 3, 1, 2), oracle.mprod(*ra, 3, 1, 2, n=n))


def test_bench_workload_full_size(ph):
    """The benchmark's matrix product at its full size: A^2 for a 3 x 3 matrix
    of degree-4 polynomials in n=8 with 300 distinct monomials each (Gaussian
    coefficients), 2,430,000 raw terms, every output term compared bitwise."""
    rng = W.rng_for(W.SEED_BASE + 95)
    n, d, terms, I = 8, 4, 300, 3
    A = [W.random_poly(rng, n, d, terms, integer=False, distinct=True) for _ in range(I * I)]
    say("mtimes: 3x3 A^2, 300-term entries (benchmark workload)")
    _case(ph, A, A, I, I, I, n, d)


def test_long_inner_dimension(ph):
    """1 x 20 by 20 x 2: each output entry gathers 20 partial products
    (18,000 raw terms, so the device-wide simplify takes them)."""
    rng = W.rng_for(3720)
    n, d = 4, 3
    A = [W.random_poly(rng, n, d, 30, integer=False) for _ in range(20)]
    B = [W.random_poly(rng, n, d, 30, integer=False) for _ in range(40)]
    say("mtimes: 1x20 by 20x2")
    _case(ph, A, B, 1, 20, 2, n, d)


def test_sum_and_prod_large_entries(ph):
    """sum along a row of four 3,000-term entries (12,000 terms per output
    entry, device-wide simplify) and prod down a column of two (each entry
    simplified to at most 210 monomials first, then one batched times)."""
    rng = W.rng_for(3721)
    n, d, R, C = 6, 4, 2, 4
    A = [W.random_poly(rng, n, d, 3000, integer=False) for _ in range(R * C)]
    a, ra = _batch(ph, A, n, d)
    say("msum: 2x4 of 3,000-term entries along dim 2")
    _same(ph, ph.msum(a, R, C, 2), oracle.msum(*ra, R, C, 2, n=n))
    say("mprod: 2x4 of 3,000-term entries along dim 1")
    _same(ph, ph.mprod(a, R, C, 1), oracle.mprod(*ra, R, C, 1, n=n))


def test_concat(ph):
    """Concatenation copies every entry unchanged, empty batches included."""
    rng = W.rng_for(3730)
    n = 3
    parts = [[W.random_poly(rng, n, 3, int(rng.integers(0, 20)), integer=False) for _ in range(k)]
             for k in (3, 0, 5, 1)]
    bs = [_batch(ph, ps, n, 3)[0] for ps in parts]
    say("concat: four batches")
    got = ph.concat(bs)
    _same(ph, got, W.csr_from_list([p for ps in parts for p in ps], n))


def test_subs_paper_example(ph):
    """Section 3.4: u(z1 + 1, z2) = 3 + 6 z1 + 3 z1^2 + 5 z2."""
    g = json.load(open(os.path.join(HERE, "golden", "worked_examples.json")))["W8_substitution"]
    n = g["n"]
    tp = lambda e: (np.array([t[1] for t in e], np.uint8).reshape(-1, n), np.array([t[0] for t in e], float))  # noqa
    u = tp(g["u"])
    q = [tp(g["z1_plus_1"]), (np.array([[0, 1]], np.uint8), np.array([1.0]))]
    pb, _ = _batch(ph, [u], n, 2)
    qb, rq = _batch(ph, q, n, 1)
    say("subs: Section 3.4 example")
    got = ph.subs(pb, qb)
    _same(ph, got, W.csr_from_list([oracle.subs(*u, *rq, n)], n))


@pytest.mark.parametrize("seed", range(3))
def test_subs_random(ph, seed):
    """p of 15 terms in three variables (exponents up to 3) with two-variable
    substitutes of four terms; Gaussian coefficients, tol on one seed."""
    rng = W.rng_for(3740 + seed)
    n, m = 3, 2
    p = W.random_poly(rng, n, 3, 15, integer=False)
    q = [W.random_poly(rng, m, 2, 4, integer=False) for _ in range(n)]
    tol = 0.25 if seed == 2 else 0.0
    pb, _ = _batch(ph, [p], n, 3)
    qb, rq = _batch(ph, q, m, 2)
    say(f"subs: random seed={seed}")
    got = ph.subs(pb, qb, tol=tol)
    _same(ph, got, W.csr_from_list([oracle.subs(*p, *rq, m, tol=tol)], m))


def test_subs_ten_variables(ph):
    """n = m = 10, deg(p) = 4, deg(q_i) = 2: the result's exponents stay within
    deg(p) * max_exp(q) = 8, so 4-bit fields suffice (40-bit keys); the
    declared bounds of the intermediate powers and partial products follow
    that, not the sum of the factors' declarations."""
    rng = W.rng_for(3760)
    n = m = 10
    p = W.random_poly(rng, n, 4, 12)
    q = [W.random_poly(rng, m, 2, 3) for _ in range(n)]
    pb, _ = _batch(ph, [p], n, 4)
    qb, rq = _batch(ph, q, m, 2)
    say("subs: n = m = 10")
    got = ph.subs(pb, qb)
    assert got.max_exp <= 8
    _same(ph, got, W.csr_from_list([oracle.subs(*p, *rq, m)], m))
