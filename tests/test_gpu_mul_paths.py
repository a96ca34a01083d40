"""times + simplify on both device paths, bit-exact against the oracle.

A single pair above the `mul_sort_min_raw` tunable goes through the global
radix sort of the raw product; smaller pairs and batches through the bucket
kernel.  Each case here runs with the sort path forced on (threshold 0) and
forced off, so both are held to the oracle on the same inputs, including
edge cases: one giant run of equal keys, keys that use all 64 bits, dropped
zeros, a device-detected exponent error."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

BIG = 1 << 62


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_06575_amd as ph
    ph.lib()
    old = ph.tune_get("mul_sort_min_raw")
    yield ph
    ph.tune_set("mul_sort_min_raw", old)


@pytest.fixture(params=["sort", "bucket"])
def path(request, ph):
    ph.tune_set("mul_sort_min_raw", 0 if request.param == "sort" else BIG)
    return request.param


def bitwise(got, rp, E, C):
    grp, gE, gC = got
    assert np.array_equal(grp, rp), "row pointers differ"
    assert np.array_equal(gE, E), "exponent rows differ"
    assert gC.view(np.uint64).tolist() == np.asarray(C, np.float64).view(np.uint64).tolist(), \
        "coefficients differ bitwise"


def run_pair(ph, aE, aC, bE, bC, n, max_exp, tol=0.0):
    a = ph.batch_from_numpy([0, aE.shape[0]], aE, aC, n=n, max_exp=max_exp)
    b = ph.batch_from_numpy([0, bE.shape[0]], bE, bC, n=n, max_exp=max_exp)
    got = ph.batch_to_numpy(ph.mul(a, b, tol=tol))
    oe, oc = oracle.mul(aE, aC, bE, bC, tol=tol)
    bitwise(got, np.array([0, oe.shape[0]]), oe, oc)
    return oe.shape[0]


def test_plain_small(ph, path):
    wl = W.plain_small()
    say(f"[{path}] plain small 200x200")
    run_pair(ph, wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs, 4, 6)


@pytest.mark.parametrize("seed", range(4))
def test_random_single_pairs(ph, path, seed):
    rng = W.rng_for(900 + seed)
    n = int(rng.integers(1, 8))
    d = int(rng.integers(1, 6))
    A = W.random_poly(rng, n, d, int(rng.integers(1, 400)), integer=bool(seed % 2))
    B = W.random_poly(rng, n, d, int(rng.integers(1, 400)), integer=bool(seed % 2))
    say(f"[{path}] random pair seed={seed} n={n} d={d} |A|={A[0].shape[0]} |B|={B[0].shape[0]}")
    run_pair(ph, A[0], A[1], B[0], B[1], n, d)


def test_several_tiles_and_ragged_tail(ph, path):
    """700 x 700 terms: 490,000 raw terms, many sort tiles and a ragged
    last tile; Gaussian coefficients, so only (i, j)-ordered sums match."""
    wl = W.plain_large(seed=W.SEED_BASE + 40, terms=700, n=6, d=6)
    say(f"[{path}] 700x700 n=6")
    run_pair(ph, wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs, 6, 6)


def test_giant_run(ph, path):
    """3000 copies of x1 times 5 copies of x2: one run of 15,000 products."""
    rng = W.rng_for(41)
    aE = np.tile(np.array([[1, 0, 0]], np.uint8), (3000, 1))
    bE = np.tile(np.array([[0, 1, 0]], np.uint8), (5, 1))
    say(f"[{path}] giant run")
    assert run_pair(ph, aE, rng.standard_normal(3000), bE, rng.standard_normal(5), 3, 1) == 1


def test_full_width_keys(ph, path):
    """n = 16 variables at 4 bits per field: packed keys use all 64 bits,
    so the last radix pass works on the top byte."""
    rng = W.rng_for(77)
    n = 16
    A = W.random_poly(rng, n, 7, 300)
    B = W.random_poly(rng, n, 7, 300)
    A[0][:, 0] = rng.integers(0, 8, A[0].shape[0])   # exercise the top field
    B[0][:, 0] = rng.integers(0, 8, B[0].shape[0])
    say(f"[{path}] 64-bit keys")
    run_pair(ph, A[0], A[1], B[0], B[1], n, 7)


def test_zero_drop_tolerance(ph, path):
    """(x + y)(x - y) = x^2 - y^2: the xy terms cancel exactly and are
    dropped; with tol = 1.5 the unit terms go too."""
    aE = np.array([[1, 0], [0, 1]], np.uint8)
    bE = np.array([[1, 0], [0, 1]], np.uint8)
    say(f"[{path}] cancellation")
    assert run_pair(ph, aE, np.array([1.0, 1.0]), bE, np.array([1.0, -1.0]), 2, 1) == 2
    assert run_pair(ph, aE, np.array([1.0, 1.0]), bE, np.array([1.0, -1.0]), 2, 1, tol=1.5) == 0


def test_device_detected_exponent_error(ph, path):
    lie = ph.batch_from_numpy([0, 1], np.array([[5, 0]], np.uint8), np.array([1.0]), n=2, max_exp=2)
    with pytest.raises(ph.PolyError) as ei:
        ph.mul(lie, lie)
    assert ei.value.code == 5


def test_long_partner(ph, path):
    """q with 9,000 terms against 40: more partners than one workgroup holds
    (the bucket path sorts its operands segment by segment)."""
    wl = W.plain_large(seed=W.SEED_BASE + 44, terms=9000, n=8, d=8)
    say(f"[{path}] 40 x 9000 n=8")
    run_pair(ph, wl.a_exps[:40], wl.a_coefs[:40], wl.b_exps, wl.b_coefs, 8, 8)


@pytest.mark.parametrize("bits", [4, 9, 10, 11])
def test_sort_digit_widths(ph, bits):
    """The global radix sorts with other widest digits (the sort_digit_bits
    tunable): fewer, wider passes -- up to 2,048 bins per tile -- must give
    the same bits: one pair with many tiles, one with 64-bit keys, and the
    device-wide simplify of a batch."""
    old_bits, old_min = ph.tune_get("sort_digit_bits"), ph.tune_get("simplify_wide_min")
    try:
        ph.tune_set("sort_digit_bits", bits)
        ph.tune_set("mul_sort_min_raw", 0)
        wl = W.plain_large(seed=W.SEED_BASE + 40, terms=700, n=6, d=6)
        say(f"[digits {bits}] 700x700 n=6")
        run_pair(ph, wl.a_exps, wl.a_coefs, wl.b_exps, wl.b_coefs, 6, 6)
        rng = W.rng_for(78)
        A = W.random_poly(rng, 16, 7, 300)
        B = W.random_poly(rng, 16, 7, 300)
        A[0][:, 0] = rng.integers(0, 8, A[0].shape[0])
        B[0][:, 0] = rng.integers(0, 8, B[0].shape[0])
        say(f"[digits {bits}] 64-bit keys")
        run_pair(ph, A[0], A[1], B[0], B[1], 16, 7)
        ph.tune_set("simplify_wide_min", 1)
        bm = W.batch_matrix(seed=W.SEED_BASE + 79, entries=60, tmin=10, tmax=5000, npts=0)
        say(f"[digits {bits}] device-wide simplify, {int(bm.row_ptr[-1])} terms")
        sb = ph.batch_from_numpy(bm.row_ptr, bm.exps, bm.coefs, n=bm.n, max_exp=bm.max_exp)
        orp, oe, oc = oracle.simplify_batch(bm.row_ptr, bm.exps, bm.coefs)
        bitwise(ph.batch_to_numpy(ph.simplify(sb)), orp, oe, oc)
    finally:
        ph.tune_set("sort_digit_bits", old_bits)
        ph.tune_set("simplify_wide_min", old_min)
