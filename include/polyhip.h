/*
 * polyhip -- C ABI of the MI355X (gfx950) sparse monomial-table algebra core.
 *
 * Operations follow "Polylab: A MATLAB Toolbox for Multivariate Polynomial
 * Modeling" (Niu & Yau):
 *   poly_mul       entrywise times followed by simplify   (Table "coresemantics"; Section 3.3)
 *   poly_simplify  merge repeated monomials, drop |s| <= tol (Table "apisignature", simplify(p,zeroprec))
 *   poly_jacobian  symbolic diff / jacobian                 (Section 3.3, diff(p,i), jacobian(p))
 *   poly_eval      value at numeric points                  (Section 3.3, p.eval(x0))
 *   poly_grad      gradient row evaluated at points         (Table "apisignature", g = jacobian(p))
 *   poly_hess      Hessian array evaluated at points        (Table "apisignature", H = jacobian(g))
 *   poly_eval_backward  reverse mode of poly_eval w.r.t. points and coefficients
 *   poly_eval_backward2 reverse mode of poly_eval_backward (Hessian-vector products)
 *   poly_eval_dense     P polynomials over one shared monomial set (coefficient
 *                       matrix times monomial-value matrix), in FP64 or in
 *                       split BF16 products with FP32 accumulation and FP64
 *                       recombination.
 *
 * Data model.  A polynomial in n variables is T terms; term t has a row of n
 * unsigned 8-bit exponents and an FP64 coefficient (the coefficient/exponent
 * constructor MPOLY(n,coef,pow), Table "apisignature").  A batch of P
 * polynomials (a polynomial matrix flattened row-major, or any list) is CSR:
 * polynomial p owns terms [row_ptr[p], row_ptr[p+1]).  Zero terms is the
 * structural zero polynomial.
 *
 * Canonical order.  Outputs of poly_mul and poly_simplify list each
 * polynomial's terms with exponent rows in ascending lexicographic order,
 * x1 most significant (the order of the paper's simplify(p+q) transcript,
 * Section 3.2).  Equal rows are merged by summing their coefficients in the
 * order the raw terms appear (for poly_mul: term i of a, then term j of b,
 * i-major) and the merged term is kept iff !(|s| <= zero_tol).
 *
 * Memory.  Every pointer is a DEVICE pointer unless its comment says [host].
 * The caller owns all memory (inputs, outputs, workspace).  The library keeps
 * no per-call state and allocates nothing on the device (its one device
 * array is the fixed scratch of poly_simplify_noalloc); every entry point
 * enqueues its kernels on `stream` (a hipStream_t passed as void*, NULL = the
 * default stream) and returns without synchronising.
 *
 * Errors.  Every entry point returns a poly_status.  Argument, shape and
 * size errors are detected on the host before any launch.  Data-dependent
 * problems found on the device (an exponent above the declared max_exp, an
 * output capacity that is too small) are recorded in the first 256 bytes of
 * the workspace; poly_read_status() synchronises the stream and returns them.
 * A launch failure returns POLY_ERR_HIP.
 */
#ifndef POLYHIP_H
#define POLYHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum poly_status {
    POLY_OK = 0,
    POLY_ERR_ARG = 1,          /* bad pointer, size or shape (host-detected)          */
    POLY_ERR_KEY_OVERFLOW = 2, /* no longer returned (keys of any width are handled)  */
    POLY_ERR_WORKSPACE = 3,    /* workspace smaller than the query returned           */
    POLY_ERR_CAPACITY = 4,     /* output capacity too small (device-detected)         */
    POLY_ERR_EXPONENT = 5,     /* an exponent exceeds the declared max_exp (device)   */
    POLY_ERR_UNSUPPORTED = 6,  /* shape beyond this library's limits                  */
    POLY_ERR_HIP = 7,          /* a HIP runtime call or kernel launch failed          */
    POLY_ERR_SCRATCH = 8       /* work needs more than the fixed scratch of an
                                  allocation-free entry point (host-detected)         */
} poly_status;

typedef enum poly_prec {
    POLY_FP64 = 0,             /* FP64 arithmetic throughout                           */
    POLY_SPLIT_BF16 = 1        /* split BF16 slices, FP32 MFMA accumulation, FP64 sum  */
} poly_prec;

/* A CSR batch of npolys polynomials, all in nvars variables.
 *   nvars        n, 1 <= n <= 255.
 *   max_exp      [host] caller's bound on every exponent stored in exps
 *                (0..255).  Packed-key widths are derived from it; a stored
 *                exponent above it is reported as POLY_ERR_EXPONENT.
 *   npolys       P >= 0.
 *   capacity     number of term slots allocated in exps / coefs.
 *   row_ptr_host [host] copy of row_ptr (P+1 entries) for inputs; the
 *                library plans launches from it and never reads row_ptr on
 *                the host.  Ignored (may be NULL) for outputs.
 *   row_ptr      [P+1] int64, row_ptr[0] = 0, nondecreasing.  Written by the
 *                library for outputs.
 *   exps         [capacity * n] uint8, row-major (term-major).
 *   coefs        [capacity] double. */
typedef struct poly_csr {
    int32_t nvars;
    int32_t max_exp;
    int64_t npolys;
    int64_t capacity;
    const int64_t *row_ptr_host;
    int64_t *row_ptr;
    uint8_t *exps;
    double *coefs;
} poly_csr;

/* Human-readable text for a status code. Never NULL. */
const char *poly_strerror(int32_t status);

/* Synchronises `stream`, then returns the device-detected status recorded in
 * the workspace `ws` by the last call that used it (POLY_OK if none). */
poly_status poly_read_status(const void *ws, void *stream);

/* -------------------------------------------------------------- tunables
 * Launch parameters chosen by the project's autotuner
 * (paper_2604_06575_amd/autotune.py, cache in paper_2604_06575_amd/tuning/).
 * Names: "mul_bucket_terms"  raw product terms per bucket workgroup (times)
 *        "mul_sort_min_raw"  raw terms from which a single pair is multiplied
 *                            by the global radix-sort path instead
 *        "seg_blocks_per_cu" persistent workgroups per CU (simplify, sort)
 *        "simplify_wide_min" largest-entry size from which simplify and mtimes
 *                            merge through the device-wide sort
 *        "eval_blocks_per_cu" point-tile workgroups per CU (sparse eval)
 *        "sort_digit_bits"   widest digit (4..11 bits) of the global radix
 *                            sorts (times of one large pair, device-wide
 *                            simplify, mtimes): fewer, wider passes
 *        "dense_f64_rows"    rows per workgroup of the FP64 dense
 *                            contraction (poly_eval_dense) and of the dC
 *                            of its reverse mode: 64 or 128
 *        "deriv_fused_max_n" largest n for which poly_grad and the dX of
 *                            poly_eval_backward stream derivatives straight
 *                            from the source terms (0: always through the
 *                            formed Jacobian)
 * poly_tune_set returns POLY_ERR_ARG for an unknown name or a value outside
 * the tunable's range; values are process-wide and apply to later calls.
 * Workspace sizes depend on them: query the workspace again after a change. */
poly_status poly_tune_set(const char *name, int64_t value);
poly_status poly_tune_get(const char *name, int64_t *value);

/* ----------------------------------------------------------- kernel timing
 * Measurement hook for benchmarks.  While enabled, the library records a
 * pair of HIP events on the caller's stream around the dominant kernel of an
 * entry point, in slots:
 *   POLY_TIMING_MUL   poly_mul: the bucketed expand + sort + merge kernel, or
 *                     on the radix-sort path each scatter pass
 *   POLY_TIMING_DENSE the contraction kernel of poly_eval_dense
 *   POLY_TIMING_TERMS the term-streaming kernel of poly_eval / grad / hess
 *   POLY_TIMING_AFFINE the per-point kernel of poly_affine_normal or
 *                     poly_affine_normal_stochastic
 * poly_timing_enable(1) clears every slot and starts recording; (0) stops.
 * poly_timing_read waits for the recorded events of `slot` (at most the last
 * 1024 launches are kept) and returns their summed duration in milliseconds
 * and the launch count.  Off by default; recording adds two event records per
 * launch and is not meant for graph capture.  Not thread-safe with concurrent
 * entry-point calls from other host threads. */
enum { POLY_TIMING_MUL = 0, POLY_TIMING_DENSE = 1, POLY_TIMING_TERMS = 2, POLY_TIMING_AFFINE = 3 };
poly_status poly_timing_enable(int32_t enable);
poly_status poly_timing_read(int32_t slot, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------- simplify
 * out_p = simplify(in_p, zero_tol) for every p (Table "coresemantics").
 * Inputs may hold repeated monomials in any order.  Batches whose largest
 * entry has fewer than "simplify_wide_min" terms are processed by one
 * persistent launch that takes entries largest first (exponent rows packed
 * into 64-bit keys of b = bit width of max_exp bits per variable, x1 in the
 * top field); otherwise by one device-wide stable radix sort of the keys
 * entry * (max_exp + 1)^n + (mixed-radix monomial key) and a tiled merge of
 * equal-key runs.  Where that key passes 64 bits it is cut into words below
 * 2^64 at variable boundaries and sorted word by word, least significant
 * first; where n*b > 64 the device-wide path is taken whatever the sizes.
 * All paths sum each run left to right in input order, so they give
 * bit-identical results.  The device-wide path needs fewer than 2^32 terms
 * in all (else POLY_ERR_UNSUPPORTED when n*b > 64; the per-entry path is
 * taken otherwise).
 * out->npolys must equal in->npolys, out->nvars in->nvars; out->capacity >=
 * total input terms always suffices.  zero_tol >= 0 (NaN sums are kept). */
poly_status poly_simplify_workspace(const poly_csr *in, size_t *ws_bytes);
poly_status poly_simplify(const poly_csr *in, poly_csr *out, double zero_tol,
                          void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------------------------------------- mul
 * out_p = simplify(a_p .* b_p, zero_tol): every term of a_p times every term
 * of b_p (exponent rows added, coefficients multiplied once, no fused
 * multiply-add), then merged as in poly_simplify (Section 3.3, entrywise
 * times; Section 6.3, expansion followed by simplify).  a and b must have
 * equal nvars and npolys.  Field width b = bit width of
 * (a->max_exp + b->max_exp) <= 8.  Per pair, |a_p| * |b_p| must be below
 * 2^32.  *raw_terms (host) receives sum_p |a_p| * |b_p|; out->capacity >=
 * that always suffices (the exact need is the final row_ptr[P]).  With
 * n*b <= 64 the raw product terms are never written to memory: they are
 * generated per key range inside the merge kernel.  With n*b > 64 they are
 * written as exponent rows in the order of the definition (sum_p |a_p| *
 * |b_p| below 2^32) and simplified over key words as in poly_simplify. */
poly_status poly_mul_workspace(const poly_csr *a, const poly_csr *b,
                               size_t *ws_bytes, int64_t *raw_terms);
poly_status poly_mul(const poly_csr *a, const poly_csr *b, poly_csr *out,
                     double zero_tol, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- jacobian
 * Symbolic Jacobian (Section 3.3): out entry p*n + j = diff(in_p, x_{j+1}).
 * A term with e_j > 0 becomes (e - u_j, c * e_j); other terms vanish; term
 * order is preserved.  out->npolys = P * n; out->capacity >= n * total input
 * terms always suffices. */
poly_status poly_jacobian_workspace(const poly_csr *in, size_t *ws_bytes);
poly_status poly_jacobian(const poly_csr *in, poly_csr *out,
                          void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------- evaluation
 * X is [N * n] row-major FP64 points.  x^0 = 1 (also 0^0); an empty
 * polynomial evaluates to 0.
 *   poly_eval: Y[p*N + pt]                = f_p(x_pt)
 *   poly_grad: G[(p*N + pt)*n + j]        = d f_p / d x_{j+1} (x_pt)
 *   poly_hess: H[((p*N + pt)*n + j)*n + k] = d^2 f_p / dx_{j+1} dx_{k+1} (x_pt),
 *              both triangles, bitwise symmetric (each Hessian entry is the
 *              polynomial with coefficient c * e_j * (e_k - [j==k]), the
 *              integer multiplier formed first).
 * Summation order inside the library is not the oracle's storage order, so
 * results agree with a sequential FP64 sum to rounding, not bitwise.
 *
 * prec selects the arithmetic (nslices is read only for the split path):
 *   POLY_FP64        term streaming in FP64 on the vector units (any batch).
 *   POLY_SPLIT_BF16  for a batch that is one shared monomial set stored as
 *       CSR -- every polynomial lists the same K exponent rows in the same
 *       order -- the coefficients are the P x K matrix of the dense split
 *       contraction of poly_eval_dense (split BF16 digits, FP32 MFMA sums,
 *       FP64 recombination; error bound as stated there), used in place.
 *       Gradients are n such contractions over the derived monomial sets
 *       e - u_j with coefficients e_j c, Hessians n (n + 1) / 2 over
 *       e - u_j - u_k with coefficients e_j (e_k - [j == k]) c (the integer
 *       multiplier formed first; entry (k, j) copied from (j, k)).  Unequal
 *       polynomial lengths: POLY_ERR_UNSUPPORTED from the call (host check);
 *       unequal rows: POLY_ERR_UNSUPPORTED in the device status (the
 *       outputs are then undefined).  The workspace query takes the same
 *       prec and nslices. */
poly_status poly_eval_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes);
poly_status poly_eval(const poly_csr *f, const double *X, int64_t N, double *Y, poly_prec prec, int32_t nslices,
                      void *ws, size_t ws_bytes, void *stream);
poly_status poly_grad_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes);
poly_status poly_grad(const poly_csr *f, const double *X, int64_t N, double *G, poly_prec prec, int32_t nslices,
                      void *ws, size_t ws_bytes, void *stream);
poly_status poly_hess_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes);
poly_status poly_hess(const poly_csr *f, const double *X, int64_t N, double *H, poly_prec prec, int32_t nslices,
                      void *ws, size_t ws_bytes, void *stream);

/* Reverse mode of Y = poly_eval(f, X) for a cotangent gY[P*N]:
 *   dC[t]        = sum_pt gY[p(t)*N + pt] * x_pt^{e_t}          (may be NULL)
 *   dX[pt*n + j] = sum_p  gY[p*N + pt] * d f_p / d x_{j+1}(x_pt) (may be NULL)
 * prec: POLY_FP64, or POLY_SPLIT_BF16 for a batch that is one shared
 * monomial set (every polynomial the same K exponent rows in the same order,
 * as for poly_eval): then the call is poly_eval_dense_backward on that set
 * with C the P x K coefficient matrix (dC and dX split on nslices digits,
 * its limits included); unequal row lengths give
 * POLY_ERR_UNSUPPORTED, unequal rows POLY_ERR_UNSUPPORTED in the status word
 * (poly_read_status). */
poly_status poly_eval_backward_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices,
                                         size_t *ws_bytes);
poly_status poly_eval_backward(const poly_csr *f, const double *X, int64_t N,
                               const double *gY, double *dX, double *dC, poly_prec prec, int32_t nslices,
                               void *ws, size_t ws_bytes, void *stream);

/* Reverse mode of poly_eval_backward (second order; what a double backward
 * of evaluation needs).  With cotangents u[N*n] of dX and w[T] of dC, and
 * L = sum_t w[t] dC[t] + sum_{pt,j} u[pt*n + j] dX[pt*n + j]:
 *   ggY[p*N + pt] = dL/dgY = sum_{t in p} (c_t sum_k u[pt*n+k] d m_t/dx_k (x_pt) + w[t] m_t(x_pt))
 *   ggX[pt*n + j] = dL/dX  = sum_t gY[p(t)*N + pt] (c_t sum_k u[pt*n+k] d2 m_t/dx_j dx_k (x_pt)
 *                                                   + w[t] d m_t/dx_j (x_pt))
 *   ggC[t]        = dL/dc  = sum_pt gY[p(t)*N + pt] sum_k u[pt*n+k] d m_t/dx_k (x_pt)
 * (m_t = x^{e_t}).  The first sum over k is a Hessian-vector product per
 * point; it is computed term by term from the monomials' second derivatives,
 * and no Hessian or derivative polynomial is formed.  u or w may be NULL
 * (taken as zero); any output may be NULL.  Limits: n <= 105 (the points,
 * the direction and one accumulator block per wave share the 160 KB LDS of a
 * workgroup), else POLY_ERR_UNSUPPORTED. */
poly_status poly_eval_backward2_workspace(const poly_csr *f, int64_t N, size_t *ws_bytes);
poly_status poly_eval_backward2(const poly_csr *f, const double *X, int64_t N, const double *gY,
                                const double *u, const double *w, double *ggY, double *ggX, double *ggC,
                                void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------------------- polynomial matrices
 * out = A * B for polynomial matrices (Section 3.3, mtimes: matrix
 * semantics): A is I x K and B is K x J CSR batches with entries in
 * row-major order (A->npolys == I*K, B->npolys == K*J, same nvars);
 * out->npolys == I*J.  Entry (i, j) is simplify(R_ij, zero_tol) where R_ij
 * concatenates, for k = 0..K-1, the raw products of A_ik and B_kj in
 * (term of A_ik, term of B_kj) order (exponent rows added, coefficients
 * multiplied and rounded once).  out->max_exp >= A->max_exp + B->max_exp
 * (at most 255); out->capacity >= the raw term count returned by the query
 * (device-checked, POLY_ERR_CAPACITY).  Matrix powers are repeated products.
 * When an output entry has at least "simplify_wide_min" raw terms and the
 * keys fit 64 bits, the raw products go straight to the device-wide
 * simplify as packed keys; otherwise they are written as exponent rows and
 * simplified as in poly_simplify (any width). */
poly_status poly_mtimes_workspace(const poly_csr *A, const poly_csr *B, int64_t I, int64_t K, int64_t J,
                                  size_t *ws_bytes, int64_t *raw_terms);
poly_status poly_mtimes(const poly_csr *A, const poly_csr *B, int64_t I, int64_t K, int64_t J,
                        poly_csr *out, double zero_tol, void *ws, size_t ws_bytes, void *stream);

/* -------------------------------------------------------- concatenation
 * out = the entries of ins[0], ins[1], ..., ins[nin-1] in order (a
 * polynomial array built from the arrays of Section 3.1; the substitution
 * of Section 3.4 gathers its power tables this way).  All inputs share
 * out->nvars and have max_exp <= out->max_exp; out->npolys == sum of npolys;
 * out->capacity >= total input terms (host-checked, POLY_ERR_CAPACITY).
 * Terms are copied unchanged; no workspace. */
poly_status poly_concat(const poly_csr *const *ins, int32_t nin, poly_csr *out, void *stream);

/* ------------------------------------------------------- affine normal
 * Affine-normal direction of one polynomial (f->npolys == 1, 2 <= n <= 255)
 * at N points (Section 5, the exact log-determinant method): with
 * g = grad f(x), e = g / |g|, an orthonormal frame Q = [Q_T, e],
 * A = Q_T' Hess f(x) Q_T + reg I, h = Q_T' Hess f(x) e and
 * a_i = tr(A^-1 Q_T' D^3 f(x)[Q_T e_i] Q_T) (i = 1..n-1):
 *   D[pt*n + i] = (Q [A^-1 (h - |g| / (n + 1) a); -1])_i
 * (independent of the choice of Q_T; the regularization reg >= 0 enters
 * every tangent solve), and gnorm[pt] = |g| (gnorm may be NULL).
 * The gradient and Hessian come from the poly_grad / poly_hess paths; the
 * third-order term is contracted per monomial, so no n^3 tensor is formed.
 * Terms of total degree above 12 are not supported (device status
 * POLY_ERR_UNSUPPORTED).  A singular regularized tangent block, or g = 0,
 * gives non-finite output for that point.  X [N*n] row-major; D [N*n].
 * Up to n = 128 each point's n x n work matrix lives in LDS; beyond, in the
 * point's Hessian slot of the workspace (the same results, HBM-bound). */
poly_status poly_affine_normal_workspace(const poly_csr *f, int64_t N, size_t *ws_bytes);
poly_status poly_affine_normal(const poly_csr *f, const double *X, int64_t N, double reg,
                               double *D, double *gnorm, void *ws, size_t ws_bytes, void *stream);

/* Affine-normal direction by the stochastic log-determinant route of
 * Section 5 (MF-logDet-Stochastic): the same direction as
 * poly_affine_normal with each trace a_i replaced by a Hutchinson average
 * over q probes and each solve with A by conjugate gradients.
 *   Z          probes in R^n, [q*n] row-major shared by all points, or
 *              [N*q*n] (point-major) when per_point = 1.  The tangent probe
 *              of Z_s is z_s = Q_T' Z_s; Rademacher Z gives an unbiased
 *              estimate of a, and sqrt(n) times an orthonormal basis of R^n
 *              (q = n) gives a exactly.
 *   a_i      ~ (1/q) sum_s D^3 f[Q_T y_s, Q_T z_s, Q_T e_i], y_s = A^-1 z_s
 *   tau        the solve of A tau = h - |g| / (n + 1) a
 *   D[pt*n+i]  (Q [tau; -1])_i, gnorm[pt] = |g|.
 * Every solve is conjugate gradients from 0 with one A-product per step,
 * taken while fewer than maxit products have been made and |r| > tol |b|
 * (a step with p'Ap = 0 ends the solve).  hv_evals[pt] (may be NULL)
 * receives the Hessian-vector products made at the point: one for H e plus
 * one per step of the q + 1 solves; the third-derivative contractions per
 * point are q.  Matrix-free: Hessian-vector products and third derivatives
 * are taken per monomial, the n x n Hessian is never formed.
 * One polynomial, 2 <= n <= 255, q >= 1, tol >= 0, maxit >= 0 with
 * (q + 1) * maxit + 1 <= 2^31 - 1 (the count fits int32), reg >= 0
 * (else POLY_ERR_ARG); terms of total degree above 12 give the device
 * status POLY_ERR_UNSUPPORTED.  g = 0 gives non-finite output for that
 * point.  X [N*n], D [N*n], gnorm [N] (required). */
poly_status poly_affine_normal_stochastic_workspace(const poly_csr *f, int64_t N, size_t *ws_bytes);
poly_status poly_affine_normal_stochastic(const poly_csr *f, const double *X, int64_t N, const double *Z,
                                          int32_t q, int32_t per_point, double reg, double tol, int32_t maxit,
                                          double *D, double *gnorm, int32_t *hv_evals, void *ws, size_t ws_bytes,
                                          void *stream);

/* ----------------------------------------------------- shared monomial set
 * Y[p*N + pt] = sum_k C[p*K + k] * prod_i X[pt*n + i]^basis[k*n + i]:
 * P polynomials over one set of K monomials (basis, [K * n] uint8), i.e. the
 * coefficient matrix C [P x K] times the monomial-value matrix V [K x N]
 * built on the fly from per-point power tables.
 *   prec = POLY_FP64:       V and the products in FP64 (FP64 MFMA).
 *   prec = POLY_SPLIT_BF16: C and V are split into `nslices` BF16 slices
 *       with a power-of-two scale per (row, K-block of 128) and (point,
 *       K-block); slice products of diagonals s + t = 2 and 3 are summed
 *       exactly in FP32 by BF16 MFMA within each K-block, diagonals >= 4
 *       share one FP32 accumulator, and each K-block is recombined in FP64.
 *       nslices in [3, 5] (a sixth digit would sit below the FP32
 *       rounding floor of the shared accumulator, so it is refused with
 *       POLY_ERR_ARG); pairs with s + t > nslices + 1 are skipped.
 * Error of the split result is about max(2^-(8*nslices - 10), 2^-34)
 * relative to sum over K-blocks b of (sum_{k in b} |C[p,k]|) * max_{k in b}
 * |v_k(x)| (digits are relative to the block's largest monomial value; this
 * equals sum_k |C v| when the values of a block share a binade): digit
 * truncation, or the FP32 rounding of the accumulator shared by digit
 * diagonals s + t >= 4.
 * Limits (POLY_ERR_UNSUPPORTED beyond them): the points of one tile and a
 * row of ones fit in LDS (n <= 94 for FP64, n <= 89 for the split
 * path at nslices = 5), and one workgroup's rows of C, or of one BF16
 * slice of C, are addressed with 32-bit byte offsets: K <= 2,097,120 for
 * FP64 with 128 rows per workgroup (the "dense_f64_rows" tunable), else
 * K <= 4,194,272.  The split digits carry their block's power-of-two scale
 * as BF16 numbers and their products are summed in FP32, so the path
 * assumes that the product of the two operands' block magnitudes (C and V;
 * gY and V, or C and gY, in the reverse mode) lies between about 2^-78 and
 * 2^126; beyond that range digit products underflow or overflow. */
poly_status poly_eval_dense_workspace(int32_t n, int64_t K, int64_t P, int64_t N,
                                      poly_prec prec, int32_t nslices, size_t *ws_bytes);
poly_status poly_eval_dense(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp,
                            int64_t P, const double *C, int64_t N, const double *X,
                            double *Y, poly_prec prec, int32_t nslices,
                            void *ws, size_t ws_bytes, void *stream);

/* Reverse mode of poly_eval_dense for a cotangent gY [P x N]:
 *   dC[p*K + k]  = sum_pt gY[p*N + pt] * v_k(x_pt)            (may be NULL)
 *   dX[pt*n + j] = sum_k W[k][pt] * d v_k / d x_{j+1} (x_pt),
 *                  W = C^T gY                                   (may be NULL)
 * prec POLY_FP64: both on FP64 MFMA.  dC with V^T formed per step of
 * points; dX per tile of 128 points, the W tile of each 64 monomials formed
 * and contracted at once with the monomials' derivatives (W never stored).
 * prec POLY_SPLIT_BF16: the forward's split scheme on nslices (3..5) BF16
 * digits per operand, FP32 sums exact per 128-long block of the
 * contraction, FP64 accumulation across blocks.  dC: digits of gY and V^T
 * scaled per 128-point block (error relative to sum_pt |gY v_k| as the
 * forward's to sum_k |C v|).  dX: W = C^T gY from digits of C^T and gY^T
 * scaled per 128-polynomial block, stored in FP64 per chunk of 4,096 points,
 * then contracted with the monomials' derivatives in FP64 (error relative to
 * sum_k sum_p |C gY| |d v_k / d x_j|).  Limits: dX needs n <= 43, split dC
 * n <= 64, and the split digit rows of one workgroup stay below 2^31 bytes
 * (N, P below about 4.19 million), else POLY_ERR_UNSUPPORTED; nslices
 * outside 3..5 with POLY_SPLIT_BF16 is POLY_ERR_ARG; basis, C and X as in
 * poly_eval_dense.  The split workspace holds the digit planes of gY, C^T
 * and gY^T (2 * nslices bytes per padded element of each), the V^T scales,
 * one W chunk (8 * K * min(N, 4096) bytes) and 16 partial dX chunks. */
poly_status poly_eval_dense_backward_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec,
                                               int32_t nslices, size_t *ws_bytes);
poly_status poly_eval_dense_backward(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P,
                                     const double *C, int64_t N, const double *X, const double *gY,
                                     double *dC, double *dX, poly_prec prec, int32_t nslices,
                                     void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ plans
 * A plan records, once, the pipeline of a polynomial matrix
 *   simplified = simplify(in, zero_tol)        (Table "coresemantics")
 *   jac        = jacobian(simplified)          (Section 3.3; entry p*n + j)
 *   G[(p*N + pt)*n + j] = value of jac entry p*n + j at x_pt
 * into one HIP graph; poly_plan_launch replays it on a stream with no host
 * work and no read-back.  Sizes the eager calls learn by reading back
 * (simplified and Jacobian term counts) stay on the device: the Jacobian is
 * formed over worst-case work items, and its encoding and evaluation stop
 * at the counts the device wrote.  Everything the plan touches is fixed at
 * creation: in (its row_ptr_host too: the simplify launch shape depends on
 * it), X, simplified, jac, G and ws must stay allocated until
 * poly_plan_destroy; their contents may change between launches (new
 * coefficients, exponents within max_exp, new points).  Requirements:
 * simplified->npolys == in->npolys, capacity >= total input terms;
 * jac->npolys == in->npolys * n, jac->capacity >= total input terms *
 * min(n, 8) (terms with more than eight variables can need more: the device
 * then reports POLY_ERR_CAPACITY); stream must not be NULL (the legacy
 * stream cannot be captured); kernel timing (poly_timing_enable) must be
 * off while a plan is created.  Device-detected errors land in the status
 * word of ws (poly_read_status).  Calls that overlap on one plan race. */
typedef struct poly_plan poly_plan;
poly_status poly_plan_workspace(const poly_csr *in, int64_t N, size_t *ws_bytes);
poly_status poly_plan_create(const poly_csr *in, double zero_tol, const double *X, int64_t N,
                             poly_csr *simplified, poly_csr *jac, double *G,
                             void *ws, size_t ws_bytes, void *stream, poly_plan **plan);
poly_status poly_plan_launch(const poly_plan *plan, void *stream);
poly_status poly_plan_destroy(poly_plan *plan);

/* ------------------------------------------------ allocation-free simplify
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * operation, kernels and results as poly_simplify (bit-identical outputs),
 * but the workspace is a fixed array of POLY_NOALLOC_SCRATCH_BYTES in device
 * memory that the library owns: one per GPU, held from the first call on
 * that GPU until the process ends.  Nothing is allocated or freed by this
 * call; the caller still owns `in` and `out`.
 *   status  [device] int32 that receives the device-detected status of the
 *           call (as poly_read_status would report it: POLY_OK,
 *           POLY_ERR_EXPONENT, POLY_ERR_CAPACITY), written by a kernel on
 *           `stream` after the last one of the call; may be NULL.
 * Returns POLY_ERR_SCRATCH, before any device work, when the workspace that
 * poly_simplify_workspace reports for `in` exceeds the fixed scratch: about
 * 24 bytes per term and 16 per polynomial on the per-entry path (some 2.7
 * million terms), about 49 bytes per term when the batch takes the
 * device-wide path (an entry of at least "simplify_wide_min" terms; some 1.3
 * million terms).
 * Every call on a GPU shares that GPU's scratch and finds it as the last call
 * left it; what the kernels need cleared they clear themselves.  Calls that
 * overlap on one GPU (from several streams or host threads) race on the
 * scratch and give undefined results: serialise them. */
#define POLY_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
poly_status poly_simplify_noalloc(const poly_csr *in, poly_csr *out, double zero_tol, int32_t *status,
                                  void *stream);

#ifdef __cplusplus
}
#endif

#endif /* POLYHIP_H */
