// Products of polynomial matrices (Section 3.3: mtimes follows matrix
// semantics).  A is I x K and B is K x J, both CSR batches with entries in
// row-major order.  Entry (i, j) of the product is simplify of the raw
// products of A_ik and B_kj concatenated over k = 0..K-1, each in (term of
// A_ik, term of B_kj) order: these kernels write that raw batch, the
// batched simplify merges it.
#include "kernels.h"

// products and sums are rounded separately, as in the definition (no FMA)
#pragma clang fp contract(off)

namespace polyhip {

// raw terms of every output entry: sizes[i * J + j] = sum_k |A_ik| |B_kj|
__global__ void k_mat_raw_sizes(const int64_t *a_rp, const int64_t *b_rp, int64_t I, int64_t K, int64_t J,
                                int64_t *sizes)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= I * J) return;
    const int64_t i = q / J, j = q % J;
    int64_t r = 0;
    for (int64_t k = 0; k < K; ++k)
        r += (a_rp[i * K + k + 1] - a_rp[i * K + k]) * (b_rp[k * J + j + 1] - b_rp[k * J + j]);
    sizes[q] = r;
}

// One workgroup per output entry (i, j): for each k, the |A_ik| x |B_kj|
// products (exponent rows added, coefficients multiplied) at
// r_rp[q] + (terms of earlier k) + a * |B_kj| + b.
__global__ void __launch_bounds__(MAT_THREADS) k_mat_expand(const int64_t *a_rp, const uint8_t *a_e, const double *a_c,
                                                           const int64_t *b_rp, const uint8_t *b_e, const double *b_c,
                                                           int64_t I, int64_t K, int64_t J, int n,
                                                           const int64_t *r_rp, uint8_t *r_e, double *r_c)
{
    const int64_t q = blockIdx.x;
    if (q >= I * J) return;
    const int64_t i = q / J, j = q % J;
    int64_t base = r_rp[q];
    for (int64_t k = 0; k < K; ++k) {
        const int64_t a0 = a_rp[i * K + k], ta = a_rp[i * K + k + 1] - a0;
        const int64_t b0 = b_rp[k * J + j], tb = b_rp[k * J + j + 1] - b0;
        const int64_t cnt = ta * tb;
        for (int64_t x = threadIdx.x; x < cnt; x += MAT_THREADS) {
            const int64_t a = x / tb, b = x % tb;
            const uint8_t *ea = a_e + (a0 + a) * n;
            const uint8_t *eb = b_e + (b0 + b) * n;
            uint8_t *er = r_e + (base + x) * n;
            for (int v = 0; v < n; ++v) er[v] = (uint8_t)(ea[v] + eb[v]);
            r_c[base + x] = a_c[a0 + a] * b_c[b0 + b];
        }
        base += cnt;
    }
}

}  // namespace polyhip

namespace polyhip {

// The same raw products for the device-wide simplify, one thread per raw
// term r: the output entry q holding r (a binary search of r_rp), then k and
// the factor pair; the term's key is q * span + ka + kb -- mixed-radix
// monomial keys with radix max_exp(A) + max_exp(B) + 1 add without carries --
// its value index r, its coefficient the product (span = radix^n, or 0 for
// a single output entry).
__global__ void k_mat_keys(const int64_t *__restrict__ a_rp, const uint64_t *__restrict__ ka,
                           const double *__restrict__ a_c, const int64_t *__restrict__ b_rp,
                           const uint64_t *__restrict__ kb, const double *__restrict__ b_c, int64_t I, int64_t K,
                           int64_t J, const int64_t *__restrict__ r_rp, int64_t R, uint64_t span,
                           uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, double *__restrict__ r_c)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int64_t Q = I * J;
    int64_t lo = 0, hi = Q;   // the last q < Q with r_rp[q] <= r
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (r_rp[mid] <= r) lo = mid;
        else hi = mid;
    }
    const int64_t q = lo, i = q / J, j = q % J;
    int64_t x = r - r_rp[q];
    int64_t a0 = 0, b0 = 0, tb = 1;
    for (int64_t k = 0; k < K; ++k) {
        a0 = a_rp[i * K + k];
        b0 = b_rp[k * J + j];
        const int64_t ta = a_rp[i * K + k + 1] - a0;
        tb = b_rp[k * J + j + 1] - b0;
        if (x < ta * tb) break;
        x -= ta * tb;
    }
    const int64_t a = x / tb, b = x - (x / tb) * tb;
    const uint64_t key = ka[a0 + a] + kb[b0 + b];
    keys[r] = (uint64_t)q * span + key;
    vals[r] = (uint32_t)r;
    r_c[r] = a_c[a0 + a] * b_c[b0 + b];
}

}  // namespace polyhip

namespace polyhip {

// One input batch of a concatenation: its P entries become output entries
// entry_off .. entry_off + P - 1, its T terms output terms term_off .. ;
// row pointers shifted by term_off (row_ptr[entry_off + P] is the next
// input's first pointer, written with the same value by both).
__global__ void k_concat_copy(const int64_t *__restrict__ rp, const uint8_t *__restrict__ exps,
                              const double *__restrict__ coefs, int64_t P, int64_t T, int n, int64_t entry_off,
                              int64_t term_off, int64_t *__restrict__ out_rp, uint8_t *__restrict__ out_exps,
                              double *__restrict__ out_coefs)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t p = i0; p <= P; p += stride) out_rp[entry_off + p] = rp[p] + term_off;
    for (int64_t t = i0; t < T; t += stride) out_coefs[term_off + t] = coefs[t];
    for (int64_t b = i0; b < T * n; b += stride) out_exps[term_off * n + b] = exps[b];
}

}  // namespace polyhip
