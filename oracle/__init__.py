"""Plain FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and the two
share no code: this package wraps ``poly_oracle.c`` (the plain definitions of
simplify, times, eval, diff and the reverse mode of eval) through ctypes, and
adds a brute-force simplify built on a Python dict as a second, independent
data structure for self-checks, the affine-normal direction of Section 5
written out in NumPy from the symbolic derivatives (the reference route and
the stochastic route: Hutchinson probes with conjugate-gradient solves), and
the polynomial-matrix operations of Section 3.3 (mtimes, sum and prod along a
dimension) and the substitution of Section 3.4, composed from simplify and
times.

Each function states the passage of the paper it follows; conventions where
the paper is silent are documented in ``poly_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "poly_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


def build_library() -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build_library()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    d = ctypes.c_double
    lib.orc_simplify.argtypes = [i32, i64, P, P, d, P, P]
    lib.orc_simplify.restype = i64
    lib.orc_expand.argtypes = [i32, i64, P, P, i64, P, P, P, P]
    lib.orc_expand.restype = i64
    lib.orc_mul.argtypes = [i32, i64, P, P, i64, P, P, d, P, P]
    lib.orc_mul.restype = i64
    lib.orc_eval_point.argtypes = [i32, i64, P, P, P]
    lib.orc_eval_point.restype = d
    lib.orc_eval_batch.argtypes = [i32, i64, P, P, P, i64, P, P]
    lib.orc_eval_batch.restype = None
    lib.orc_eval_dense.argtypes = [i32, i64, P, i64, P, i64, P, P]
    lib.orc_eval_dense.restype = None
    lib.orc_eval_dense_ld.argtypes = [i32, i64, P, i64, P, i64, P, P, P]
    lib.orc_eval_dense_ld.restype = None
    lib.orc_eval_batch_ld.argtypes = [i32, i64, P, P, P, i64, P, P, P]
    lib.orc_eval_batch_ld.restype = None
    lib.orc_diff.argtypes = [i32, i64, P, P, i32, P, P]
    lib.orc_diff.restype = i64
    lib.orc_diff2.argtypes = [i32, i64, P, P, i32, i32, P, P]
    lib.orc_diff2.restype = i64
    lib.orc_grad_batch.argtypes = [i32, i64, P, P, P, i64, P, P]
    lib.orc_grad_batch.restype = i32
    lib.orc_hess_batch.argtypes = [i32, i64, P, P, P, i64, P, P]
    lib.orc_hess_batch.restype = i32
    lib.orc_eval_backward.argtypes = [i32, i64, P, P, P, i64, P, P, P, P]
    lib.orc_eval_backward.restype = i32
    _lib = lib
    return lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u8(e, n):
    return np.ascontiguousarray(np.asarray(e, dtype=np.uint8).reshape(-1, n))


def _f64(c):
    return np.ascontiguousarray(np.asarray(c, dtype=np.float64).ravel())


def _check(rc: int):
    if rc == -1:
        raise MemoryError("oracle allocation failed")
    if rc == -2:
        raise OverflowError("exponent sum exceeds 255")
    if rc < 0:
        raise RuntimeError(f"oracle error {rc}")


# --------------------------------------------------------------------- simplify

def simplify(exps, coefs, tol: float = 0.0, n: int | None = None):
    """``simplify(p, zeroprec)`` (Table "coresemantics"; Table "apisignature"):
    merge repeated monomials and drop coefficients with |s| <= tol.  Output in
    canonical order (lex, x1 most significant, ascending)."""
    n = n if n is not None else np.asarray(exps).shape[1]
    e = _u8(exps, n)
    c = _f64(coefs)
    t = e.shape[0]
    oe = np.empty((max(t, 1), n), dtype=np.uint8)
    oc = np.empty(max(t, 1), dtype=np.float64)
    r = _load().orc_simplify(n, t, _p(e), _p(c), float(tol), _p(oe), _p(oc))
    _check(r)
    return oe[:r].copy(), oc[:r].copy()


def simplify_batch(row_ptr, exps, coefs, tol: float = 0.0, n: int | None = None):
    """simplify applied entrywise to a CSR batch (a polynomial matrix is an
    array of scalar objects, Section 2.1 / 3.1)."""
    n = n if n is not None else np.asarray(exps).shape[1]
    rp = np.asarray(row_ptr, dtype=np.int64)
    e = _u8(exps, n)
    c = _f64(coefs)
    outs = []
    for p in range(rp.shape[0] - 1):
        outs.append(simplify(e[rp[p]:rp[p + 1]], c[rp[p]:rp[p + 1]], tol, n))
    return _csr(outs, n)


def brute_simplify(exps, coefs, tol: float = 0.0):
    """Second, independent simplify: a dict keyed by the exponent tuple,
    accumulated in storage order, emitted in tuple order (Python's tuple
    comparison is lexicographic with the first variable most significant)."""
    acc: dict[tuple, float] = {}
    for row, c in zip(np.asarray(exps).tolist(), np.asarray(coefs, dtype=np.float64).tolist()):
        k = tuple(row)
        if k in acc:
            acc[k] = acc[k] + c
        else:
            acc[k] = c
    keys = sorted(k for k, s in acc.items() if not (abs(s) <= tol))
    n = np.asarray(exps).shape[1]
    e = np.array(keys, dtype=np.uint8).reshape(-1, n)
    c = np.array([acc[k] for k in keys], dtype=np.float64)
    return e, c


# ------------------------------------------------------------------------ times

def expand(ae, ac, be, bc, n: int | None = None):
    """Raw product terms, i-major (entrywise ``times``, Section 3.3)."""
    n = n if n is not None else np.asarray(ae).shape[1]
    ae, be = _u8(ae, n), _u8(be, n)
    ac, bc = _f64(ac), _f64(bc)
    raw = ae.shape[0] * be.shape[0]
    re = np.empty((max(raw, 1), n), dtype=np.uint8)
    rc = np.empty(max(raw, 1), dtype=np.float64)
    r = _load().orc_expand(n, ae.shape[0], _p(ae), _p(ac), be.shape[0], _p(be), _p(bc), _p(re), _p(rc))
    _check(r)
    return re[:raw].copy(), rc[:raw].copy()


def mul(ae, ac, be, bc, tol: float = 0.0, n: int | None = None):
    """``simplify(a .* b)``: expand every pair of terms, then simplify."""
    n = n if n is not None else np.asarray(ae).shape[1]
    ae, be = _u8(ae, n), _u8(be, n)
    ac, bc = _f64(ac), _f64(bc)
    raw = ae.shape[0] * be.shape[0]
    oe = np.empty((max(raw, 1), n), dtype=np.uint8)
    oc = np.empty(max(raw, 1), dtype=np.float64)
    r = _load().orc_mul(n, ae.shape[0], _p(ae), _p(ac), be.shape[0], _p(be), _p(bc), float(tol), _p(oe), _p(oc))
    _check(r)
    return oe[:r].copy(), oc[:r].copy()


def mul_batch(a_rp, a_e, a_c, b_rp, b_e, b_c, tol: float = 0.0, n: int | None = None):
    """Entrywise ``times`` over two CSR batches of equal length."""
    n = n if n is not None else np.asarray(a_e).shape[1]
    a_e, b_e = _u8(a_e, n), _u8(b_e, n)
    a_c, b_c = _f64(a_c), _f64(b_c)
    outs = []
    for p in range(len(a_rp) - 1):
        outs.append(mul(a_e[a_rp[p]:a_rp[p + 1]], a_c[a_rp[p]:a_rp[p + 1]],
                        b_e[b_rp[p]:b_rp[p + 1]], b_c[b_rp[p]:b_rp[p + 1]], tol, n))
    return _csr(outs, n)


def _csr(polys, n):
    rp = np.zeros(len(polys) + 1, dtype=np.int64)
    for i, (e, _c) in enumerate(polys):
        rp[i + 1] = rp[i] + e.shape[0]
    E = np.vstack([e for e, _ in polys]).astype(np.uint8) if polys else np.zeros((0, n), np.uint8)
    C = np.concatenate([c for _, c in polys]) if polys else np.zeros(0)
    return rp, E.reshape(-1, n), C


# ------------------------------------------------------------------------- eval

def eval_points(exps, coefs, X, n: int | None = None) -> np.ndarray:
    """``p.eval(x0)`` at each row of X (Section 3.3)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = n if n is not None else X.shape[1]
    e, c = _u8(exps, n), _f64(coefs)
    rp = np.array([0, e.shape[0]], dtype=np.int64)
    return eval_batch(rp, e, c, X)[0]


def eval_batch(row_ptr, exps, coefs, X) -> np.ndarray:
    """Y[p, pt] for every polynomial of a CSR batch at every point."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    e, c = _u8(exps, n), _f64(coefs)
    P = rp.shape[0] - 1
    Y = np.empty((P, X.shape[0]), dtype=np.float64)
    _load().orc_eval_batch(n, P, _p(rp), _p(e), _p(c), X.shape[0], _p(X), _p(Y))
    return Y


def eval_batch_ld(row_ptr, exps, coefs, X):
    """Extended-precision (80-bit) evaluation; returns (Y, sum_t |c_t v_t|)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    e, c = _u8(exps, n), _f64(coefs)
    P = rp.shape[0] - 1
    Y = np.empty((P, X.shape[0]))
    A = np.empty((P, X.shape[0]))
    _load().orc_eval_batch_ld(n, P, _p(rp), _p(e), _p(c), X.shape[0], _p(X), _p(Y), _p(A))
    return Y, A


def eval_dense(basis, C, X) -> np.ndarray:
    """Y = C V for a shared monomial set: Y[p, pt] = sum_k C[p,k] x_pt^basis_k."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    b = _u8(basis, n)
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    P, K = C.shape
    assert K == b.shape[0]
    Y = np.empty((P, X.shape[0]))
    _load().orc_eval_dense(n, K, _p(b), P, _p(C), X.shape[0], _p(X), _p(Y))
    return Y


def eval_dense_ld(basis, C, X):
    """Extended-precision twin of eval_dense; returns (Y, sum_k |C v|)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    b = _u8(basis, n)
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    P, K = C.shape
    Y = np.empty((P, X.shape[0]))
    A = np.empty((P, X.shape[0]))
    _load().orc_eval_dense_ld(n, K, _p(b), P, _p(C), X.shape[0], _p(X), _p(Y), _p(A))
    return Y, A


# ------------------------------------------------------------------ derivatives

def diff(exps, coefs, j: int, n: int | None = None):
    """``diff(p, j)`` with 0-based j (Section 3.3)."""
    n = n if n is not None else np.asarray(exps).shape[1]
    e, c = _u8(exps, n), _f64(coefs)
    oe = np.empty((max(e.shape[0], 1), n), dtype=np.uint8)
    oc = np.empty(max(e.shape[0], 1))
    r = _load().orc_diff(n, e.shape[0], _p(e), _p(c), j, _p(oe), _p(oc))
    return oe[:r].copy(), oc[:r].copy()


def diff2(exps, coefs, j: int, k: int, n: int | None = None):
    """Hessian entry (j,k) as a polynomial, integer multiplier formed first."""
    n = n if n is not None else np.asarray(exps).shape[1]
    e, c = _u8(exps, n), _f64(coefs)
    oe = np.empty((max(e.shape[0], 1), n), dtype=np.uint8)
    oc = np.empty(max(e.shape[0], 1))
    r = _load().orc_diff2(n, e.shape[0], _p(e), _p(c), j, k, _p(oe), _p(oc))
    return oe[:r].copy(), oc[:r].copy()


def jacobian_batch(row_ptr, exps, coefs, n: int | None = None):
    """``jacobian`` of a polynomial vector/matrix flattened to a CSR batch:
    output entry (p, j) = diff(f_p, j), laid out p-major then j."""
    n = n if n is not None else np.asarray(exps).shape[1]
    rp = np.asarray(row_ptr, dtype=np.int64)
    e, c = _u8(exps, n), _f64(coefs)
    outs = []
    for p in range(rp.shape[0] - 1):
        for j in range(n):
            outs.append(diff(e[rp[p]:rp[p + 1]], c[rp[p]:rp[p + 1]], j, n))
    return _csr(outs, n)


def grad_batch(row_ptr, exps, coefs, X) -> np.ndarray:
    """G[p, pt, j] = d f_p / d x_j at x_pt (jacobian then eval)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    e, c = _u8(exps, n), _f64(coefs)
    P = rp.shape[0] - 1
    G = np.empty((P, X.shape[0], n))
    _check(_load().orc_grad_batch(n, P, _p(rp), _p(e), _p(c), X.shape[0], _p(X), _p(G)))
    return G


def hess_batch(row_ptr, exps, coefs, X) -> np.ndarray:
    """H[p, pt, j, k] = d^2 f_p / dx_j dx_k at x_pt, both triangles."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    e, c = _u8(exps, n), _f64(coefs)
    P = rp.shape[0] - 1
    H = np.empty((P, X.shape[0], n, n))
    _check(_load().orc_hess_batch(n, P, _p(rp), _p(e), _p(c), X.shape[0], _p(X), _p(H)))
    return H


def eval_backward(row_ptr, exps, coefs, X, gY, want_dX: bool = True, want_dC: bool = True):
    """Reverse mode of Y = eval(f, X) for the cotangent gY[p, pt]:
    dC[t] = sum_pt gY[p(t), pt] v_t(x_pt); dX[pt, j] = sum_p gY[p, pt] df_p/dx_j."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    e, c = _u8(exps, n), _f64(coefs)
    gY = np.ascontiguousarray(np.asarray(gY, dtype=np.float64))
    P = rp.shape[0] - 1
    dX = np.empty((X.shape[0], n)) if want_dX else None
    dC = np.empty(e.shape[0]) if want_dC else None
    _check(_load().orc_eval_backward(n, P, _p(rp), _p(e), _p(c), X.shape[0], _p(X), _p(gY), _p(dX), _p(dC)))
    return dX, dC


def eval_backward2(row_ptr, exps, coefs, X, gY, u=None, w=None):
    """Reverse mode of ``eval_backward``: for cotangents u[pt, j] of dX and
    w[t] of dC, with L = <w, dC> + <u, dX>,
        ggY[p, pt] = sum_j u[pt, j] df_p/dx_j (x_pt) + f_p^w(x_pt),
        ggX[pt, j] = sum_p gY[p, pt] (sum_k d2f_p/dx_j dx_k (x_pt) u[pt, k] + df_p^w/dx_j (x_pt)),
        ggC[t]     = sum_pt gY[p(t), pt] sum_j u[pt, j] d m_t/dx_j (x_pt),
    where f^w is f with coefficients w and m_t the monomial of term t.  Every
    derivative is the symbolically differentiated polynomial evaluated at the
    point (grad_batch, hess_batch; ggC from the gradients of the one-term
    polynomials m_t).  u or w may be None (zero)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    e, c = _u8(exps, n), _f64(coefs)
    gY = np.asarray(gY, dtype=np.float64)
    P, N, T = rp.shape[0] - 1, X.shape[0], e.shape[0]
    ggY = np.zeros((P, N))
    ggX = np.zeros((N, n))
    ggC = np.zeros(T)
    if u is not None:
        u = np.asarray(u, dtype=np.float64)
        G = grad_batch(rp, e, c, X)                                  # [P, N, n]
        H = hess_batch(rp, e, c, X)                                  # [P, N, n, n]
        ggY += np.einsum("pnj,nj->pn", G, u)
        ggX += np.einsum("pn,pnjk,nk->nj", gY, H, u)
        Gt = grad_batch(np.arange(T + 1), e, np.ones(T), X)          # [T, N, n]: gradients of the monomials
        owner = np.repeat(np.arange(P), np.diff(rp))
        ggC += np.einsum("tn,tnj,nj->t", gY[owner], Gt, u)
    if w is not None:
        w = _f64(w)
        ggY += eval_batch(rp, e, w, X)
        ggX += np.einsum("pn,pnj->nj", gY, grad_batch(rp, e, w, X))
    return ggY, ggX, ggC


# ------------------------------------------------------------- affine normal

def derivatives_at(exps, coefs, x, n: int | None = None):
    """Gradient g[j], Hessian H[j, k] and third-derivative tensor T[j, k, l]
    of one polynomial at one point, each entry the evaluation of the
    symbolically differentiated polynomial (diff, diff2 and a further diff:
    the automatic-differentiation reference route of Section 5)."""
    x = np.asarray(x, dtype=np.float64)
    n = n if n is not None else x.shape[0]
    X = x[None, :]
    g = np.empty(n)
    H = np.empty((n, n))
    T = np.empty((n, n, n))
    for j in range(n):
        e1, c1 = diff(exps, coefs, j, n)
        g[j] = eval_points(e1, c1, X, n)[0] if e1.shape[0] else 0.0
        for k in range(n):
            e2, c2 = diff2(exps, coefs, j, k, n)
            H[j, k] = eval_points(e2, c2, X, n)[0] if e2.shape[0] else 0.0
            for l in range(n):
                e3, c3 = diff(e2, c2, l, n) if e2.shape[0] else (e2, c2)
                T[j, k, l] = eval_points(e3, c3, X, n)[0] if e3.shape[0] else 0.0
    return g, H, T


def tangent_frame(g):
    """An orthonormal frame Q = [Q_T, e] with last column e = g / |g| (any
    completion: the direction does not depend on it)."""
    g = np.asarray(g, dtype=np.float64)
    n = g.shape[0]
    e = g / np.linalg.norm(g)
    # QR of [e, I] gives an orthonormal basis whose first vector is +-e
    Qf, _ = np.linalg.qr(np.column_stack([e, np.eye(n)]))
    Qf = Qf[:, :n]
    if Qf[:, 0] @ e < 0:
        Qf[:, 0] = -Qf[:, 0]
    return np.column_stack([Qf[:, 1:], Qf[:, 0]])


def affine_normal_from_derivatives(g, H, T, reg: float = 0.0, Q=None):
    """Affine-normal direction of Section 5 from the derivatives at a point:
    e = g/|g|, Q = [Q_T, e], H_T = Q_T' H Q_T + reg I (the regularized
    tangent block, used in every tangent solve), h = Q_T' H e,
    a_i = tr(H_T^-1 d_{t_i} H_T) with d_{t_i} H_T = Q_T' D^3f[t_i] Q_T and
    t_i = Q_T e_i, tau = H_T^-1 (h - |g| / (n + 1) a), nu = Q [tau; -1]."""
    g = np.asarray(g, dtype=np.float64)
    n = g.shape[0]
    gn = np.linalg.norm(g)
    if Q is None:
        Q = tangent_frame(g)
    QT, e = Q[:, :n - 1], Q[:, n - 1]
    HT = QT.T @ H @ QT + reg * np.eye(n - 1)
    h = QT.T @ H @ e
    a = np.empty(n - 1)
    for i in range(n - 1):
        D3 = np.tensordot(T, QT[:, i], axes=([2], [0]))    # D^3 f [t_i], an n x n matrix
        a[i] = np.trace(np.linalg.solve(HT, QT.T @ D3 @ QT))
    tau = np.linalg.solve(HT, h - gn / (n + 1) * a)
    return Q @ np.concatenate([tau, [-1.0]]), gn


def affine_normal(exps, coefs, X, reg: float = 0.0):
    """D[pt] = affine-normal direction of one polynomial at each point of X
    (Section 5, the 'ad' reference route); also |grad f| per point."""
    X = np.asarray(X, dtype=np.float64)
    N, n = X.shape
    D = np.empty((N, n))
    gn = np.empty(N)
    for p in range(N):
        g, H, T = derivatives_at(exps, coefs, X[p], n)
        D[p], gn[p] = affine_normal_from_derivatives(g, H, T, reg)
    return D, gn


def conjugate_gradients(A, b, tol: float, maxit: int):
    """Krylov solve of A y = b for a symmetric A by conjugate gradients
    (Hestenes-Stiefel), the linear solver of the stochastic route of
    Section 5.  From y = 0, r = p = b, each step takes one product A p:
    alpha = r'r / p'Ap, y += alpha p, r -= alpha A p, p = r + (r'r)_new /
    (r'r) p.  A step is taken while fewer than maxit products have been
    made and |r| > tol |b|; a product with p'Ap = 0 ends the iteration
    (breakdown).  Returns y and the number of products."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    y = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    bn = float(np.sqrt(b @ b))
    k = 0
    while k < maxit and np.sqrt(rr) > tol * bn:
        q = A @ p
        k += 1
        pq = float(p @ q)
        if pq == 0.0:
            break
        alpha = rr / pq
        y = y + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return y, k


def third_contraction(exps, coefs, x, u, v, n: int | None = None):
    """c[l] = D^3 f(x)[u, v, e_l] = sum_jk d^3 f / dx_j dx_k dx_l (x) u_j v_k,
    taken as the Hessian of the polynomial psi = sum_j u_j d f / dx_j
    (symbolic diff, coefficients scaled by u_j) applied to v."""
    x = np.asarray(x, dtype=np.float64)
    n = n if n is not None else x.shape[0]
    pe, pc = [], []
    for j in range(n):
        if u[j] == 0.0:
            continue
        e1, c1 = diff(exps, coefs, j, n)
        pe.append(e1)
        pc.append(u[j] * c1)
    if not pe or sum(e.shape[0] for e in pe) == 0:
        return np.zeros(n)
    pe, pc = np.concatenate(pe), np.concatenate(pc)
    Hp = hess_batch(np.array([0, pe.shape[0]], np.int64), pe, pc, x[None, :])[0, 0]
    return Hp @ np.asarray(v, dtype=np.float64)


def affine_normal_stochastic(exps, coefs, X, Z, reg: float, tol: float, maxit: int):
    """Affine-normal directions by the stochastic log-det route of Section 5
    (MF-logDet-Stochastic): the traces a_i = tr(A^-1 d_{t_i} H_T) of the
    exact route are replaced by Hutchinson estimates over q probes and every
    solve with A = H_T + reg I by conjugate gradients.

    Probes are given in R^n, Z [q, n] (shared by all points) or [N, q, n];
    the tangent probe of Z_s at a point is z_s = Q_T' Z_s.  With
    y_s = A^-1 z_s (a Krylov solve) and A symmetric,
      a_i ~ (1/q) sum_s z_s' A^-1 d_{t_i} H_T z_s
          = (1/q) sum_s D^3 f[Q_T y_s, Q_T z_s, t_i],
    so a = Q_T' w with w = (1/q) sum_s D^3 f[Q_T y_s, Q_T z_s, .]; then
    tau = A^-1 (h - |g| / (n + 1) a) (another Krylov solve) and
    nu = Q [tau; -1].  Returns D [N, n], |grad f| [N] and the Hessian-vector
    products per point (one for h, one per conjugate-gradient step); the
    third-derivative contractions per point are q."""
    X = np.asarray(X, dtype=np.float64)
    N, n = X.shape
    Z = np.asarray(Z, dtype=np.float64)
    q = Z.shape[-2]
    D = np.empty((N, n))
    gn = np.empty(N)
    hv = np.zeros(N, dtype=np.int64)
    rp = np.array([0, np.asarray(exps).shape[0]], np.int64)
    for pt in range(N):
        x = X[pt]
        g = grad_batch(rp, exps, coefs, x[None, :])[0, 0]
        H = hess_batch(rp, exps, coefs, x[None, :])[0, 0]
        gn[pt] = np.linalg.norm(g)
        Q = tangent_frame(g)
        QT, e = Q[:, :n - 1], Q[:, n - 1]
        A = QT.T @ H @ QT + reg * np.eye(n - 1)
        h = QT.T @ (H @ e)
        hv[pt] = 1
        Zp = Z[pt] if Z.ndim == 3 else Z
        w = np.zeros(n)
        for s in range(q):
            z = QT.T @ Zp[s]
            y, k = conjugate_gradients(A, z, tol, maxit)
            hv[pt] += k
            w += third_contraction(exps, coefs, x, QT @ y, QT @ z, n)
        w /= q
        a = QT.T @ w
        tau, k = conjugate_gradients(A, h - gn[pt] / (n + 1) * a, tol, maxit)
        hv[pt] += k
        D[pt] = Q @ np.concatenate([tau, [-1.0]])
    return D, gn, hv


# ------------------------------------------------------- polynomial matrices

def mtimes(a_rp, a_e, a_c, b_rp, b_e, b_c, I: int, K: int, J: int, tol: float = 0.0, n: int | None = None):
    """Matrix product of polynomial matrices (Section 3.3: mtimes follows
    matrix semantics; entries row-major in CSR batches, A is I x K, B is
    K x J).  Entry (i, j) is simplify of the raw products of A_ik and B_kj
    concatenated over k = 0..K-1, each in (term of A_ik, term of B_kj)
    order; one rounding per product, the sums of simplify in that order."""
    a_rp = np.asarray(a_rp, np.int64)
    b_rp = np.asarray(b_rp, np.int64)
    n = n if n is not None else np.asarray(a_e).shape[1]
    a_e, a_c = _u8(a_e, n), _f64(a_c)
    b_e, b_c = _u8(b_e, n), _f64(b_c)
    outs = []
    for i in range(I):
        for j in range(J):
            es, cs = [], []
            for k in range(K):
                pa, pb = i * K + k, k * J + j
                e, c = expand(a_e[a_rp[pa]:a_rp[pa + 1]], a_c[a_rp[pa]:a_rp[pa + 1]],
                              b_e[b_rp[pb]:b_rp[pb + 1]], b_c[b_rp[pb]:b_rp[pb + 1]], n)
                es.append(e)
                cs.append(c)
            e = np.vstack(es) if es else np.zeros((0, n), np.uint8)
            c = np.concatenate(cs) if cs else np.zeros(0)
            outs.append(simplify(e, c, tol, n) if e.shape[0] else (e, c))
    return _csr(outs, n)


def _entries(rp, e, c, n):
    rp = np.asarray(rp, np.int64)
    e, c = _u8(e, n), _f64(c)
    return [(e[rp[p]:rp[p + 1]], c[rp[p]:rp[p + 1]]) for p in range(rp.shape[0] - 1)]


def _along(R: int, C: int, dim: int):
    """Index lists of the entries reduced into each output entry of an R x C
    matrix (row-major): dim 1 gives a 1 x C result (down each column), dim 2
    an R x 1 result (along each row)."""
    if dim == 1:
        return [[i * C + j for i in range(R)] for j in range(C)]
    if dim == 2:
        return [[i * C + j for j in range(C)] for i in range(R)]
    raise ValueError("dim must be 1 or 2")


def msum(rp, e, c, R: int, C: int, dim: int, tol: float = 0.0, n: int | None = None):
    """sum(A, dim) of an R x C polynomial matrix (Section 3.3): each output
    entry is simplify of the terms of the reduced entries concatenated in
    index order (entries as stored); an empty dimension gives structural
    zeros."""
    n = n if n is not None else np.asarray(e).shape[1]
    ents = _entries(rp, e, c, n)
    outs = []
    for idx in _along(R, C, dim):
        es = [ents[q][0] for q in idx]
        cs = [ents[q][1] for q in idx]
        ee = np.vstack(es) if es else np.zeros((0, n), np.uint8)
        cc = np.concatenate(cs) if cs else np.zeros(0)
        outs.append(simplify(ee, cc, tol, n) if ee.shape[0] else (ee, cc))
    return _csr(outs, n)


def mprod(rp, e, c, R: int, C: int, dim: int, tol: float = 0.0, n: int | None = None):
    """prod(A, dim) of an R x C polynomial matrix (Section 3.3): each output
    entry is the left fold of times (expand, then simplify) over the
    simplified reduced entries in index order, ((A_1 A_2) A_3) ...; one
    entry gives its simplified self, an empty dimension the constant 1."""
    n = n if n is not None else np.asarray(e).shape[1]
    ents = _entries(rp, e, c, n)
    outs = []
    for idx in _along(R, C, dim):
        if not idx:
            outs.append((np.zeros((1, n), np.uint8), np.ones(1)))
            continue
        acc = simplify(*ents[idx[0]], tol, n)
        for q in idx[1:]:
            acc = mul(acc[0], acc[1], *simplify(*ents[q], tol, n), tol=tol, n=n)
        outs.append(acc)
    return _csr(outs, n)


def subs(pe, pc, q_rp, q_e, q_c, m: int, tol: float = 0.0):
    """Substitution p(q_1(z), ..., q_n(z)) (Section 3.4; the worked example
    u(z1 + 1, z2)): p is one polynomial in n variables (exponent rows pe,
    coefficients pc), q a batch of n polynomials in m variables.  q_i^0 = 1,
    q_i^1 = q_i and q_i^k = simplify(q_i^(k-1) q_i); each term t forms
    acc = 1, then acc = simplify(acc * simplify(q_i^(e_ti))) for i = 1..n;
    the result is simplify of the terms' acc, each coefficient multiplied by
    c_t, concatenated in term order."""
    pe = np.asarray(pe, np.uint8)
    n = pe.shape[1]
    pc = _f64(pc)
    qs = _entries(q_rp, q_e, q_c, m)
    one = (np.zeros((1, m), np.uint8), np.ones(1))

    def power(i, k):
        if k == 0:
            return one
        acc = qs[i]
        for _ in range(k - 1):
            acc = mul(acc[0], acc[1], qs[i][0], qs[i][1], tol=tol, n=m)
        return acc

    es, cs = [], []
    for t in range(pe.shape[0]):
        acc = one
        for i in range(n):
            f = simplify(*power(i, int(pe[t, i])), tol, m)
            acc = mul(acc[0], acc[1], f[0], f[1], tol=tol, n=m)
        es.append(acc[0])
        cs.append(pc[t] * acc[1])
    if not es:
        return np.zeros((0, m), np.uint8), np.zeros(0)
    e, c = np.vstack(es), np.concatenate(cs)
    return simplify(e, c, tol, m) if e.shape[0] else (e, c)
