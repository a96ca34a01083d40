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
