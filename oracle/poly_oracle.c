/*
 * Plain FP64 CPU oracle for the sparse monomial-table algebra core of
 * "Polylab: A MATLAB Toolbox for Multivariate Polynomial Modeling".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library: it is the plain definition of each operation written out,
 * slow on purpose, in the order a reader can check against the paper.
 *
 * Data model (Table "apisignature", the coefficient/exponent constructor):
 * a polynomial in n variables is T terms; term t has a row of n unsigned
 * exponents e[t*n .. t*n+n-1] and a double coefficient c[t].
 *
 * Conventions where the paper leaves a choice (each is also listed with its
 * reason in the design notes):
 *   - canonical order: exponent rows compared lexicographically with x1 most
 *     significant, ascending.  This reproduces the only explicit simplify
 *     output the paper prints (Section 3.2, simplify(p+q)) and the printed
 *     derivative g1 (Section 3.3).
 *   - simplify (Table "coresemantics": merges repeated monomials and removes
 *     coefficients below a tolerance): stable sort, then each group of equal
 *     rows is summed left to right in that stable order; a group is kept iff
 *     !(|s| <= tol), so NaN survives and tol = 0 drops exact zeros only.
 *     A polynomial whose terms all cancel has zero terms (structural zero,
 *     Section 3.1 / prod(A,2) = [x1; 0] in Section 3.3).
 *   - times (entrywise product, Section 3.3): raw terms in i-major order
 *     (for each term of a, every term of b), exponent rows added, coefficient
 *     c_a * c_b rounded once (compiled with -ffp-contract=off), then simplify.
 *   - eval (Section 3.3, p(1,2,3) = 3): per term v = product over variables
 *     with e_i > 0 of x_i^e_i, the power formed by repeated multiplication
 *     left to right; x^0 = 1 (also 0^0); y = sum of c_t * v_t in storage
 *     order starting from 0.  An empty polynomial evaluates to 0.
 *   - diff (Section 3.3, diff(p,i), jacobian): a term with e_j > 0 becomes
 *     (e - u_j, c * e_j); other terms vanish; storage order is kept.
 *   - Hessian entry (j,k) (jacobian(jacobian(p)), Table "apisignature"):
 *     coefficient c * m with the integer m = e_j * (e_k - [j==k]) formed
 *     first, exponent row e - u_j - u_k.  Entry (j,k) and (k,j) are then the
 *     same polynomial, bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ALLOC -1
#define ORC_ERR_EXP_OVERFLOW -2

/* ------------------------------------------------------------------ order */

static int row_cmp(const uint8_t *a, const uint8_t *b, int n)
{
    for (int i = 0; i < n; ++i) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

/* Stable top-down merge sort of an index permutation by row_cmp. */
static void merge_sort(int64_t *idx, int64_t *tmp, int64_t lo, int64_t hi,
                       const uint8_t *e, int n)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    merge_sort(idx, tmp, lo, mid, e, n);
    merge_sort(idx, tmp, mid, hi, e, n);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        /* take from the left run on ties: stability */
        if (row_cmp(e + idx[j] * n, e + idx[i] * n, n) < 0) tmp[k++] = idx[j++];
        else tmp[k++] = idx[i++];
    }
    while (i < mid) tmp[k++] = idx[i++];
    while (j < hi) tmp[k++] = idx[j++];
    memcpy(idx + lo, tmp + lo, (size_t)(hi - lo) * sizeof(int64_t));
}

/* --------------------------------------------------------------- simplify */

/* Returns the number of output terms written to (oe, oc), or a negative
 * error.  Output is in canonical ascending order. oe/oc may hold t terms. */
int64_t orc_simplify(int n, int64_t t, const uint8_t *e, const double *c,
                     double tol, uint8_t *oe, double *oc)
{
    if (t == 0) return 0;
    int64_t *idx = (int64_t *)malloc((size_t)t * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)t * sizeof(int64_t));
    if (!idx || !tmp) { free(idx); free(tmp); return ORC_ERR_ALLOC; }
    for (int64_t i = 0; i < t; ++i) idx[i] = i;
    merge_sort(idx, tmp, 0, t, e, n);
    int64_t out = 0;
    int64_t g = 0;
    while (g < t) {
        int64_t h = g + 1;
        while (h < t && row_cmp(e + idx[h] * n, e + idx[g] * n, n) == 0) ++h;
        double s = c[idx[g]];
        for (int64_t k = g + 1; k < h; ++k) s = s + c[idx[k]];
        if (!(fabs(s) <= tol)) {
            memcpy(oe + out * n, e + idx[g] * n, (size_t)n);
            oc[out] = s;
            ++out;
        }
        g = h;
    }
    free(idx);
    free(tmp);
    return out;
}

/* ------------------------------------------------------------------ times */

/* Raw i-major expansion of a*b into (re, rc), each ta*tb terms. */
int64_t orc_expand(int n, int64_t ta, const uint8_t *ea, const double *ca,
                   int64_t tb, const uint8_t *eb, const double *cb,
                   uint8_t *re, double *rc)
{
    int64_t r = 0;
    for (int64_t i = 0; i < ta; ++i) {
        for (int64_t j = 0; j < tb; ++j) {
            for (int v = 0; v < n; ++v) {
                int s = (int)ea[i * n + v] + (int)eb[j * n + v];
                if (s > 255) return ORC_ERR_EXP_OVERFLOW;
                re[r * n + v] = (uint8_t)s;
            }
            rc[r] = ca[i] * cb[j];
            ++r;
        }
    }
    return r;
}

/* simplify(a .* b).  oe/oc must hold ta*tb terms. */
int64_t orc_mul(int n, int64_t ta, const uint8_t *ea, const double *ca,
                int64_t tb, const uint8_t *eb, const double *cb, double tol,
                uint8_t *oe, double *oc)
{
    int64_t raw = ta * tb;
    if (raw == 0) return 0;
    uint8_t *re = (uint8_t *)malloc((size_t)raw * (size_t)n);
    double *rc = (double *)malloc((size_t)raw * sizeof(double));
    if (!re || !rc) { free(re); free(rc); return ORC_ERR_ALLOC; }
    int64_t r = orc_expand(n, ta, ea, ca, tb, eb, cb, re, rc);
    if (r >= 0) r = orc_simplify(n, raw, re, rc, tol, oe, oc);
    free(re);
    free(rc);
    return r;
}

/* ------------------------------------------------------------------- eval */

static double power_rep(double x, int k)
{
    /* x^k for k >= 1 by k-1 multiplications, left to right */
    double p = x;
    for (int m = 1; m < k; ++m) p = p * x;
    return p;
}

static double monomial_value(int n, const uint8_t *row, const double *x)
{
    double v = 1.0;
    for (int i = 0; i < n; ++i) {
        if (row[i] > 0) v = v * power_rep(x[i], row[i]);
    }
    return v;
}

double orc_eval_point(int n, int64_t t, const uint8_t *e, const double *c,
                      const double *x)
{
    double y = 0.0;
    for (int64_t k = 0; k < t; ++k) y = y + c[k] * monomial_value(n, e + k * n, x);
    return y;
}

/* Batch of P polynomials in CSR (rp[P+1]) at npts points; Y[p*npts + pt]. */
void orc_eval_batch(int n, int64_t P, const int64_t *rp, const uint8_t *e,
                    const double *c, int64_t npts, const double *X, double *Y)
{
    for (int64_t p = 0; p < P; ++p) {
        int64_t t0 = rp[p], t1 = rp[p + 1];
        for (int64_t pt = 0; pt < npts; ++pt)
            Y[p * npts + pt] = orc_eval_point(n, t1 - t0, e + t0 * n, c + t0, X + pt * n);
    }
}

/* Shared monomial set (K rows of basis) with coefficient matrix C[P*K]:
 * Y[p*npts + pt] = sum_k C[p,k] * v_k(x_pt), summed over k in order. */
void orc_eval_dense(int n, int64_t K, const uint8_t *basis, int64_t P,
                    const double *C, int64_t npts, const double *X, double *Y)
{
    double *v = (double *)malloc((size_t)(K > 0 ? K : 1) * sizeof(double));
    for (int64_t pt = 0; pt < npts; ++pt) {
        for (int64_t k = 0; k < K; ++k) v[k] = monomial_value(n, basis + k * n, X + pt * n);
        for (int64_t p = 0; p < P; ++p) {
            double y = 0.0;
            for (int64_t k = 0; k < K; ++k) y = y + C[p * K + k] * v[k];
            Y[p * npts + pt] = y;
        }
    }
    free(v);
}

/* Extended-precision twin of the evaluation (x86 80-bit long double) used to
 * attribute the rounding error of FP64 results. */
static long double power_rep_ld(long double x, int k)
{
    long double p = x;
    for (int m = 1; m < k; ++m) p = p * x;
    return p;
}

void orc_eval_dense_ld(int n, int64_t K, const uint8_t *basis, int64_t P,
                       const double *C, int64_t npts, const double *X, double *Y,
                       double *absY)
{
    long double *v = (long double *)malloc((size_t)(K > 0 ? K : 1) * sizeof(long double));
    for (int64_t pt = 0; pt < npts; ++pt) {
        for (int64_t k = 0; k < K; ++k) {
            long double val = 1.0L;
            for (int i = 0; i < n; ++i) {
                int ex = basis[k * n + i];
                if (ex > 0) val = val * power_rep_ld((long double)X[pt * n + i], ex);
            }
            v[k] = val;
        }
        for (int64_t p = 0; p < P; ++p) {
            long double y = 0.0L, a = 0.0L;
            for (int64_t k = 0; k < K; ++k) {
                long double term = (long double)C[p * K + k] * v[k];
                y = y + term;
                a = a + fabsl(term);
            }
            Y[p * npts + pt] = (double)y;
            if (absY) absY[p * npts + pt] = (double)a;
        }
    }
    free(v);
}

void orc_eval_batch_ld(int n, int64_t P, const int64_t *rp, const uint8_t *e,
                       const double *c, int64_t npts, const double *X, double *Y,
                       double *absY)
{
    for (int64_t p = 0; p < P; ++p) {
        for (int64_t pt = 0; pt < npts; ++pt) {
            long double y = 0.0L, a = 0.0L;
            for (int64_t t = rp[p]; t < rp[p + 1]; ++t) {
                long double val = 1.0L;
                for (int i = 0; i < n; ++i) {
                    int ex = e[t * n + i];
                    if (ex > 0) val = val * power_rep_ld((long double)X[pt * n + i], ex);
                }
                long double term = (long double)c[t] * val;
                y = y + term;
                a = a + fabsl(term);
            }
            Y[p * npts + pt] = (double)y;
            if (absY) absY[p * npts + pt] = (double)a;
        }
    }
}

/* ------------------------------------------------------------ derivatives */

/* d/dx_j (0-based j).  Output holds at most t terms; returns the count. */
int64_t orc_diff(int n, int64_t t, const uint8_t *e, const double *c, int j,
                 uint8_t *oe, double *oc)
{
    int64_t out = 0;
    for (int64_t k = 0; k < t; ++k) {
        int ej = e[k * n + j];
        if (ej == 0) continue;
        memcpy(oe + out * n, e + k * n, (size_t)n);
        oe[out * n + j] = (uint8_t)(ej - 1);
        oc[out] = c[k] * (double)ej;
        ++out;
    }
    return out;
}

/* Hessian entry (j,k): coefficient c*m with integer m = e_j*(e_k - [j==k]). */
int64_t orc_diff2(int n, int64_t t, const uint8_t *e, const double *c, int j, int k,
                  uint8_t *oe, double *oc)
{
    int64_t out = 0;
    for (int64_t r = 0; r < t; ++r) {
        int ej = e[r * n + j];
        int ek = e[r * n + k];
        int m = ej * (ek - (j == k ? 1 : 0));
        if (m <= 0) continue;
        memcpy(oe + out * n, e + r * n, (size_t)n);
        oe[out * n + j] = (uint8_t)(oe[out * n + j] - 1);
        oe[out * n + k] = (uint8_t)(oe[out * n + k] - 1);
        oc[out] = c[r] * (double)m;
        ++out;
    }
    return out;
}

/* G[(p*npts + pt)*n + j] = (d f_p / d x_j)(x_pt). */
int orc_grad_batch(int n, int64_t P, const int64_t *rp, const uint8_t *e,
                   const double *c, int64_t npts, const double *X, double *G)
{
    int64_t tmax = 0;
    for (int64_t p = 0; p < P; ++p) if (rp[p + 1] - rp[p] > tmax) tmax = rp[p + 1] - rp[p];
    uint8_t *de = (uint8_t *)malloc((size_t)(tmax > 0 ? tmax : 1) * (size_t)n);
    double *dc = (double *)malloc((size_t)(tmax > 0 ? tmax : 1) * sizeof(double));
    if (!de || !dc) { free(de); free(dc); return ORC_ERR_ALLOC; }
    for (int64_t p = 0; p < P; ++p) {
        int64_t t0 = rp[p], t = rp[p + 1] - rp[p];
        for (int j = 0; j < n; ++j) {
            int64_t dt = orc_diff(n, t, e + t0 * n, c + t0, j, de, dc);
            for (int64_t pt = 0; pt < npts; ++pt)
                G[(p * npts + pt) * n + j] = orc_eval_point(n, dt, de, dc, X + pt * n);
        }
    }
    free(de);
    free(dc);
    return ORC_OK;
}

/* H[((p*npts + pt)*n + j)*n + k] = (d^2 f_p / dx_j dx_k)(x_pt), both triangles. */
int orc_hess_batch(int n, int64_t P, const int64_t *rp, const uint8_t *e,
                   const double *c, int64_t npts, const double *X, double *H)
{
    int64_t tmax = 0;
    for (int64_t p = 0; p < P; ++p) if (rp[p + 1] - rp[p] > tmax) tmax = rp[p + 1] - rp[p];
    uint8_t *de = (uint8_t *)malloc((size_t)(tmax > 0 ? tmax : 1) * (size_t)n);
    double *dc = (double *)malloc((size_t)(tmax > 0 ? tmax : 1) * sizeof(double));
    if (!de || !dc) { free(de); free(dc); return ORC_ERR_ALLOC; }
    for (int64_t p = 0; p < P; ++p) {
        int64_t t0 = rp[p], t = rp[p + 1] - rp[p];
        for (int j = 0; j < n; ++j) {
            for (int k = 0; k < n; ++k) {
                int64_t dt = orc_diff2(n, t, e + t0 * n, c + t0, j, k, de, dc);
                for (int64_t pt = 0; pt < npts; ++pt)
                    H[((p * npts + pt) * n + j) * n + k] =
                        orc_eval_point(n, dt, de, dc, X + pt * n);
            }
        }
    }
    free(de);
    free(dc);
    return ORC_OK;
}

/* Reverse mode of Y[p,pt] = f_p(x_pt) for a cotangent gY[p*npts+pt]:
 *   dC[t]            = sum over pt of gY[p(t),pt] * v_t(x_pt)     (pt ascending)
 *   dX[pt*n + j]     = sum over p of gY[p,pt] * (d f_p/dx_j)(x_pt) (p ascending)
 * Either output may be NULL. */
int orc_eval_backward(int n, int64_t P, const int64_t *rp, const uint8_t *e,
                      const double *c, int64_t npts, const double *X,
                      const double *gY, double *dX, double *dC)
{
    if (dC) {
        for (int64_t p = 0; p < P; ++p) {
            for (int64_t t = rp[p]; t < rp[p + 1]; ++t) {
                double s = 0.0;
                for (int64_t pt = 0; pt < npts; ++pt)
                    s = s + gY[p * npts + pt] * monomial_value(n, e + t * n, X + pt * n);
                dC[t] = s;
            }
        }
    }
    if (dX) {
        double *G = (double *)malloc((size_t)(P * npts * n > 0 ? P * npts * n : 1) * sizeof(double));
        if (!G) return ORC_ERR_ALLOC;
        int rc = orc_grad_batch(n, P, rp, e, c, npts, X, G);
        if (rc != ORC_OK) { free(G); return rc; }
        for (int64_t pt = 0; pt < npts; ++pt) {
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int64_t p = 0; p < P; ++p)
                    s = s + gY[p * npts + pt] * G[(p * npts + pt) * n + j];
                dX[pt * n + j] = s;
            }
        }
        free(G);
    }
    return ORC_OK;
}
