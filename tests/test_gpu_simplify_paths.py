"""simplify and mtimes on both device paths, bit-exact against the oracle.

A batch whose largest polynomial has at least `simplify_wide_min` terms is
simplified by one device-wide radix sort of (polynomial, monomial) keys and a
tiled run merge; other batches by one workgroup per polynomial.  Each case
runs with the device-wide path forced on (threshold 1) and forced off, so both
are held to the oracle on the same inputs: runs that cross merge tiles and the
halo, empty polynomials between full ones, cancellation to the structural
zero, keys that use all 64 bits, dropped terms, a device-detected exponent
error."""
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
    old = ph.tune_get("simplify_wide_min")
    yield ph
    ph.tune_set("simplify_wide_min", old)


@pytest.fixture(params=["wide", "per_poly"])
def path(request, ph):
    ph.tune_set("simplify_wide_min", BIG if request.param == "per_poly" else 1)
    return request.param


def bitwise(got, rp, E, C):
    grp, gE, gC = got
    assert np.array_equal(grp, rp), "row pointers differ"
    assert np.array_equal(gE, E), "exponent rows differ"
    assert gC.view(np.uint64).tolist() == np.asarray(C, np.float64).view(np.uint64).tolist(), \
        "coefficients differ bitwise"


def run_batch(ph, polys, n, max_exp, tol=0.0):
    rp, E, C = W.csr_from_list(polys, n)
    got = ph.batch_to_numpy(ph.simplify(ph.batch_from_numpy(rp, E, C, n=n, max_exp=max_exp), tol))
    bitwise(got, *oracle.simplify_batch(rp, E, C, tol, n=n))
    return got


@pytest.mark.parametrize("seed", range(4))
def test_random_batches(ph, path, seed):
    """Up to 30 polynomials of up to 3,000 terms (several 2,048-element merge
    tiles), some empty, repeated monomials in random order."""
    rng = W.rng_for(5100 + seed)
    n = int(rng.integers(1, 7))
    d = int(rng.integers(1, 6))
    P = int(rng.integers(1, 30))
    polys = []
    for _ in range(P):
        t = 0 if rng.random() < 0.2 else int(rng.integers(1, 3000))
        polys.append(W.random_poly(rng, n, d, t, integer=bool(seed % 2)))
    tol = 0.0 if seed < 2 else 0.5
    say(f"[{path}] simplify seed={seed} n={n} d={d} P={P} T={sum(p[0].shape[0] for p in polys)}")
    run_batch(ph, polys, n, d, tol)


def test_runs_across_tiles(ph, path):
    """One monomial repeated 9,000 times (a run through several tiles, past
    the halo), a run that cancels exactly, and empty polynomials around."""
    rng = W.rng_for(5201)
    e = np.tile(np.array([[1, 2, 0]], np.uint8), (9000, 1))
    c = rng.standard_normal(9000)
    mixed = W.random_poly(rng, 3, 3, 4000)
    e2 = np.vstack([mixed[0][:2000], e[:3000], mixed[0][2000:]])
    c2 = np.concatenate([mixed[1][:2000], c[:3000], mixed[1][2000:]])
    cancel = (np.tile(np.array([[0, 1, 1]], np.uint8), (4000, 1)), np.tile(np.array([1.5, -1.5]), 2000))
    z = (np.zeros((0, 3), np.uint8), np.zeros(0))
    polys = [z, (e, c), z, z, (e2, c2), cancel, z]
    say(f"[{path}] runs across tiles")
    got = run_batch(ph, polys, 3, 3)
    assert got[0][6] - got[0][5] == 0   # the cancelled entry is the structural zero


def test_full_width_keys(ph, path):
    """n=8 with exponents up to 255: monomial keys use all 64 bits, so the
    device-wide path takes a single polynomial only; two polynomials fall
    back to the per-polynomial path on either setting."""
    rng = W.rng_for(5202)
    base = rng.integers(0, 256, size=(700, 8)).astype(np.uint8)
    E = base[rng.integers(0, 700, size=6000)]
    C = rng.standard_normal(6000)
    say(f"[{path}] 64-bit keys, one polynomial")
    run_batch(ph, [(E, C)], 8, 255)
    say(f"[{path}] 64-bit keys, two polynomials")
    run_batch(ph, [(E[:3000], C[:3000]), (E[3000:], C[3000:])], 8, 255)


def test_single_key_value(ph, path):
    """max_exp 0: every key is the polynomial index alone."""
    polys = [(np.zeros((5000, 2), np.uint8), np.full(5000, 0.25)), (np.zeros((3, 2), np.uint8), np.ones(3))]
    say(f"[{path}] max_exp 0")
    run_batch(ph, polys, 2, 0)


def test_device_detected_exponent_error(ph, path):
    lie = ph.batch_from_numpy([0, 1], np.array([[5, 0]], np.uint8), np.array([1.0]), n=2, max_exp=2)
    with pytest.raises(ph.PolyError) as ei:
        ph.simplify(lie)
    assert ei.value.code == 5


def _mat(ph, polys, n, d):
    rp, E, C = W.csr_from_list(polys, n)
    return ph.batch_from_numpy(rp, E, C, n=n, max_exp=d), (rp, E, C)


@pytest.mark.parametrize("I,K,J,terms", [(3, 3, 3, 60), (2, 5, 1, 90), (1, 1, 1, 150)])
def test_mtimes(ph, path, I, K, J, terms):
    """Entries of up to `terms` random monomials: several merge tiles per
    output entry; Gaussian coefficients, so the summation order matters."""
    rng = W.rng_for(5300 + I + 10 * K + 100 * J)
    n, d = 4, 3
    A = [W.random_poly(rng, n, d, int(rng.integers(0, terms)), integer=False) for _ in range(I * K)]
    B = [W.random_poly(rng, n, d, int(rng.integers(0, terms)), integer=False) for _ in range(K * J)]
    a, ra = _mat(ph, A, n, d)
    b, rb = _mat(ph, B, n, d)
    say(f"[{path}] mtimes {I}x{K} by {K}x{J}, up to {terms} terms")
    got = ph.batch_to_numpy(ph.mtimes(a, b, I, K, J))
    bitwise(got, *oracle.mtimes(*ra, *rb, I, K, J, n=n))


def test_mtimes_tolerance(ph, path):
    rng = W.rng_for(5310)
    n, d = 2, 3
    A = [W.random_poly(rng, n, d, 40) for _ in range(4)]
    a, ra = _mat(ph, A, n, d)
    say(f"[{path}] mtimes with tol")
    got = ph.batch_to_numpy(ph.mtimes(a, a, 2, 2, 2, tol=200.0))
    bitwise(got, *oracle.mtimes(*ra, *ra, 2, 2, 2, tol=200.0, n=n))
