"""Seeded synthetic inputs for the sparse monomial-table algebra core.

This module only *draws* inputs: exponent tables, coefficients and points, with
the shapes and distributions of the workloads described for the paper's
benchmarks (Table "benchmeta", Section 6.1) and of the five scaled-up
workloads this library is measured on.  It holds none of the method's
arithmetic (no products, sorting of terms, merging or evaluation), so the
oracle under ``oracle/`` and the HIP path can both consume it without sharing
any computation.

Conventions
-----------
* A polynomial is a pair ``(exps, coefs)``: ``exps`` is a ``uint8`` array of
  shape ``[T, n]`` (row = monomial, column = variable, the coefficient/exponent
  constructor of Table "apisignature"), ``coefs`` is ``float64[T]``.
* A batch is CSR: ``row_ptr`` (``int64[P+1]``), ``exps`` (``uint8[T, n]``),
  ``coefs`` (``float64[T]``).
* Points are ``float64[N, n]`` row-major.
* Every generator takes an integer ``seed`` and uses ``numpy`` PCG64.
  The default seeds follow the paper's convention of fixed seeds
  (20260321, 20260322; Section 6.1): workload ``k`` uses ``20260321 + k``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 20260321


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Monomial sets
# ---------------------------------------------------------------------------

def basis(n: int, d: int) -> np.ndarray:
    """All exponent vectors in ``n`` variables of total degree <= ``d``.

    Count is C(n+d, d) (Section 3.1, the ``monolist`` count).  Rows are
    produced by recursion on the first variable; no particular order is
    promised to consumers.
    """
    if n < 1 or d < 0:
        raise ValueError("need n >= 1 and d >= 0")
    # rows[k] = all vectors over the last m variables with total degree <= k
    rows = [np.arange(k + 1, dtype=np.int64)[:, None] for k in range(d + 1)]
    for _m in range(2, n + 1):
        nxt = []
        for k in range(d + 1):
            parts = []
            for e in range(k + 1):
                tail = rows[k - e]
                head = np.full((tail.shape[0], 1), e, dtype=np.int64)
                parts.append(np.hstack([head, tail]))
            nxt.append(np.vstack(parts))
        rows = nxt
    out = rows[d].astype(np.uint8)
    assert out.shape[0] == math.comb(n + d, d)
    return out


def _stars_and_bars(rng: np.random.Generator, n: int, d: int, m: int) -> np.ndarray:
    """``m`` exponent vectors drawn uniformly over all monomials of degree <= d.

    A monomial with |alpha| <= d is a composition of d into n+1 parts (the last
    part is slack), i.e. a choice of d "star" slots among n+d.  A uniform
    d-subset of slots therefore gives a uniform monomial.
    """
    slots = n + d
    out = np.zeros((0, n), dtype=np.uint8)
    while out.shape[0] < m:
        want = (m - out.shape[0]) * 2 + 16
        s = rng.integers(0, slots, size=(want, d))
        s.sort(axis=1)
        if d > 1:
            ok = np.all(np.diff(s, axis=1) > 0, axis=1)
            s = s[ok]
        part = s - np.arange(d)[None, :]          # part index of each star, 0..n
        e = np.zeros((s.shape[0], n + 1), dtype=np.int64)
        rows = np.repeat(np.arange(s.shape[0]), d)
        np.add.at(e, (rows, part.ravel()), 1)
        out = np.vstack([out, e[:, :n].astype(np.uint8)])
    return out[:m]


def _row_ids(exps: np.ndarray) -> np.ndarray:
    """Opaque per-row identity used only for de-duplicating draws."""
    return np.ascontiguousarray(exps).view(np.dtype((np.void, exps.shape[1]))).ravel()


def distinct_monomials(rng: np.random.Generator, n: int, d: int, m: int) -> np.ndarray:
    """``m`` distinct monomials, uniform over all monomials of degree <= d."""
    total = math.comb(n + d, d)
    if m > total:
        raise ValueError(f"only {total} monomials of degree <= {d} in {n} variables")
    if total <= 2_000_000:
        b = basis(n, d)
        idx = rng.choice(total, size=m, replace=False)
        return b[idx]
    got = np.zeros((0, n), dtype=np.uint8)
    while got.shape[0] < m:
        cand = np.vstack([got, _stars_and_bars(rng, n, d, (m - got.shape[0]) * 11 // 10 + 8)])
        _, first = np.unique(_row_ids(cand), return_index=True)
        got = cand[np.sort(first)]
    return got[:m]


def monomials_with_replacement(rng: np.random.Generator, n: int, d: int, m: int) -> np.ndarray:
    """``m`` monomials drawn independently and uniformly (repeats allowed)."""
    return _stars_and_bars(rng, n, d, m)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclass
class PairWorkload:
    n: int
    a_exps: np.ndarray
    a_coefs: np.ndarray
    b_exps: np.ndarray
    b_coefs: np.ndarray
    max_exp: int          # bound on any exponent of the two operands
    X: np.ndarray | None  # evaluation points (or None)


def plain_small(seed: int = SEED_BASE + 1, npts: int = 1024) -> PairWorkload:
    """Two random sparse polynomials in n=4 variables of degree <= 6, 200
    distinct terms each, integer coefficients uniform on {-9..9} (zero
    included), plus ``npts`` points uniform in [-1,1]^4."""
    rng = rng_for(seed)
    n, d, t = 4, 6, 200
    ae = distinct_monomials(rng, n, d, t)
    be = distinct_monomials(rng, n, d, t)
    ac = rng.integers(-9, 10, size=t).astype(np.float64)
    bc = rng.integers(-9, 10, size=t).astype(np.float64)
    X = rng.uniform(-1.0, 1.0, size=(npts, n))
    return PairWorkload(n, ae, ac, be, bc, d, X)


def plain_large(seed: int = SEED_BASE + 2, terms: int = 5000, n: int = 10, d: int = 8) -> PairWorkload:
    """p and q in n=10 variables of degree <= 8 with 5,000 distinct terms
    each and N(0,1) coefficients; the product has degree <= 16 and
    ``terms**2`` raw terms."""
    rng = rng_for(seed)
    ae = distinct_monomials(rng, n, d, terms)
    be = distinct_monomials(rng, n, d, terms)
    ac = rng.standard_normal(terms)
    bc = rng.standard_normal(terms)
    return PairWorkload(n, ae, ac, be, bc, d, None)


@dataclass
class BatchWorkload:
    n: int
    row_ptr: np.ndarray
    exps: np.ndarray
    coefs: np.ndarray
    max_exp: int
    X: np.ndarray | None


def batch_matrix(seed: int = SEED_BASE + 3, entries: int = 4096, n: int = 20, d: int = 6,
                 tmin: int = 10, tmax: int = 20000, npts: int = 4096) -> BatchWorkload:
    """A polynomial matrix (64 x 64 = 4,096 entries by default) in n=20
    variables of degree <= 6.  Entry term counts are log-uniform on
    [tmin, tmax]; each entry's terms are drawn uniformly over the monomials
    with replacement, so entries hold repeated monomials in random order;
    N(0,1) coefficients; points uniform in [-1,1]^n."""
    rng = rng_for(seed)
    counts = np.floor(np.exp(rng.uniform(math.log(tmin), math.log(tmax), size=entries))).astype(np.int64)
    counts = np.clip(counts, tmin, tmax)
    row_ptr = np.zeros(entries + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    total = int(row_ptr[-1])
    exps = monomials_with_replacement(rng, n, d, total)
    coefs = rng.standard_normal(total)
    X = rng.uniform(-1.0, 1.0, size=(npts, n)) if npts else None
    return BatchWorkload(n, row_ptr, exps, coefs, d, X)


@dataclass
class DenseWorkload:
    n: int
    basis: np.ndarray     # [K, n] shared monomial set
    C: np.ndarray         # [P, K] coefficient matrix
    X: np.ndarray         # [N, n] points


def dense_shared(seed: int = SEED_BASE + 4, P: int = 4096, N: int = 65536, n: int = 30, d: int = 4,
                 K: int | None = None) -> DenseWorkload:
    """``P`` polynomials over a shared monomial set, N(0,1) coefficient matrix
    and ``N`` points uniform in [-1,1]^n.  At n=30, degree <= 4 the set is the
    full basis (C(34,4) = 46,376 monomials; fewer exist than the 50,000 the
    workload description names).  ``K`` < full basis takes a random subset."""
    rng = rng_for(seed)
    b = basis(n, d)
    if K is not None and K < b.shape[0]:
        b = b[np.sort(rng.choice(b.shape[0], size=K, replace=False))]
    C = rng.standard_normal((P, b.shape[0]))
    X = rng.uniform(-1.0, 1.0, size=(N, n))
    return DenseWorkload(n, b, C, X)


@dataclass
class ScalarWorkload:
    n: int
    exps: np.ndarray
    coefs: np.ndarray
    X: np.ndarray


def quartic(seed: int = SEED_BASE + 5, n: int = 100, terms: int = 100_000, npts: int = 8192,
            d: int = 4) -> ScalarWorkload:
    """A random quartic: ``terms`` distinct monomials uniform over degree <= 4
    in ``n`` variables, N(0,1) coefficients, points uniform in [-1,1]^n."""
    rng = rng_for(seed)
    e = distinct_monomials(rng, n, d, terms)
    c = rng.standard_normal(terms)
    X = rng.uniform(-1.0, 1.0, size=(npts, n))
    return ScalarWorkload(n, e, c, X)


def sparse_quartic(seed: int = SEED_BASE + 6, n: int = 64, npts: int = 4096, m: int | None = None,
                   support: int = 3) -> ScalarWorkload:
    """The affine-normal timing families: ``m`` distinct quartic monomials of
    support size 3 (default m = 4n; exponents a permutation of (2, 1, 1) on
    three distinct variables) or of support size 2 (default m = 3n;
    exponents (a, 4 - a) on two distinct variables, a uniform in {1, 2, 3}),
    N(0,1) coefficients, plus sum_i x_i^2 so the tangent Hessian blocks stay
    nonsingular; points uniform in [-1,1]^n."""
    if support not in (2, 3):
        raise ValueError("support must be 2 or 3")
    rng = rng_for(seed)
    m = (4 * n if support == 3 else 3 * n) if m is None else m
    rows, seen = [], set()
    while len(rows) < m:
        v = rng.choice(n, size=support, replace=False)
        e = np.zeros(n, dtype=np.uint8)
        if support == 3:
            e[v] = (2, 1, 1)
        else:
            a = int(rng.integers(1, 4))
            e[v] = (a, 4 - a)
        key = e.tobytes()
        if key not in seen:
            seen.add(key)
            rows.append(e)
    E = np.vstack(rows + [2 * np.eye(n, dtype=np.uint8)])
    C = np.concatenate([rng.standard_normal(m), np.ones(n)])
    X = rng.uniform(-1.0, 1.0, size=(npts, n))
    return ScalarWorkload(n, E, C, X)


def homogeneous(seed: int, n: int, d: int, terms: int, coef_range: int = 5) -> tuple[np.ndarray, np.ndarray]:
    """Distinct monomials of total degree exactly ``d`` with small integer
    coefficients (for Euler-identity checks)."""
    rng = rng_for(seed)
    pool = basis(n, d)
    pool = pool[pool.astype(np.int64).sum(axis=1) == d]
    terms = min(terms, pool.shape[0])
    e = pool[rng.choice(pool.shape[0], size=terms, replace=False)]
    c = rng.integers(-coef_range, coef_range + 1, size=terms).astype(np.float64)
    c[c == 0] = 1.0
    return e, c


def all_ones_family(n: int, d: int) -> tuple[np.ndarray, np.ndarray]:
    """p_d = sum over all monomials of degree <= d, every coefficient 1
    (the heavy-simplify family of Section 6.3)."""
    e = basis(n, d)
    return e, np.ones(e.shape[0], dtype=np.float64)


def random_poly(rng: np.random.Generator, n: int, d: int, terms: int, integer: bool = True,
                distinct: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Small random polynomial for fuzz cases (repeats allowed unless distinct)."""
    if terms == 0:
        return np.zeros((0, n), dtype=np.uint8), np.zeros(0, dtype=np.float64)
    if distinct:
        e = distinct_monomials(rng, n, d, min(terms, math.comb(n + d, d)))
    else:
        e = monomials_with_replacement(rng, n, d, terms)
    if integer:
        c = rng.integers(-9, 10, size=e.shape[0]).astype(np.float64)
    else:
        c = rng.standard_normal(e.shape[0])
    return e, c


def points(seed: int, npts: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng_for(seed).uniform(lo, hi, size=(npts, n))


def integer_points(seed: int, npts: int, n: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    return rng_for(seed).integers(lo, hi + 1, size=(npts, n)).astype(np.float64)


def csr_from_list(polys: list[tuple[np.ndarray, np.ndarray]], n: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Concatenate a list of (exps, coefs) into CSR arrays."""
    rp = np.zeros(len(polys) + 1, dtype=np.int64)
    for i, (e, _c) in enumerate(polys):
        rp[i + 1] = rp[i] + e.shape[0]
    if polys:
        E = np.vstack([e.reshape(-1, n) for e, _ in polys]).astype(np.uint8)
        C = np.concatenate([c for _, c in polys]).astype(np.float64)
    else:
        E = np.zeros((0, n), dtype=np.uint8)
        C = np.zeros(0, dtype=np.float64)
    return rp, E, C
