// Simplify of batches that hold large polynomials (Section 3.1: sort the
// terms of each polynomial by monomial, combine equal monomials, drop the
// zeros), as one device-wide sort instead of one workgroup per polynomial.
//
// Each term gets the key p * r^n + sum_i e_i r^(n-1-i) (polynomial p, radix
// r = max_exp + 1, x1 the most significant digit), so one stable LSD radix
// sort over the whole batch orders every polynomial's terms by monomial, the
// polynomials one after another, and equal monomials in their input order;
// mixed-radix digits keep the key range, and so the number of passes, as
// small as the exponent bound allows.  The merge then sums each run of equal
// keys left to right (the order of the definition, so results are
// bit-identical to the per-polynomial path) and stages the kept terms with
// their exponents as bit fields for the unpack kernel; the row pointers come
// from binary searches of the sorted keys.
#include "kernels.h"

namespace polyhip {

// span = r^n, or 0 for a single polynomial
__global__ void k_ws_keys(const uint8_t *__restrict__ exps, int64_t T, int n, uint32_t radix, int max_exp,
                          const int64_t *__restrict__ row_ptr, int64_t P, uint64_t span, uint64_t *__restrict__ keys,
                          uint32_t *__restrict__ vals, int32_t *status)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint8_t *row = exps + t * n;
    uint64_t k = 0;
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t e = row[i];
        bad |= (int)(e > (uint32_t)max_exp);
        k = k * radix + e;
    }
    // the polynomial holding term t: the last p < P with row_ptr[p] <= t
    int64_t lo = 0, hi = P;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (row_ptr[mid] <= t) lo = mid;
        else hi = mid;
    }
    keys[t] = (uint64_t)lo * span + k;
    vals[t] = (uint32_t)t;
    if (bad) set_status(status, POLY_ERR_EXPONENT);
}

// Tiles of MG_TILE sorted elements; persistent workgroups take tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...  The run heads of a tile are
// compacted and each lane sums one run left to right from LDS; the tile's
// last run continues through a halo of GS_HALO elements and, past that, the
// sorted stream itself.  Runs whose head lies in an earlier tile belong to
// that tile.  Kept sums are staged in element order at [b * MG_TILE, ...)
// with their composite keys (st_ckey) and their exponents as bit fields of
// `bits` bits, x1 in the top field (st_key, the unpack kernel's layout).
__global__ void __launch_bounds__(MG_THREADS) k_ws_merge(const uint64_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ vals, int64_t R,
                                                        const double *__restrict__ coefs, double tol,
                                                        uint64_t span, uint32_t radix, int n, int bits,
                                                        uint64_t *__restrict__ st_key, uint64_t *__restrict__ st_ckey,
                                                        double *__restrict__ st_coef, int64_t *seg_count,
                                                        int64_t *stage_off)
{
    __shared__ uint64_t s_key[MG_TILE + GS_HALO];
    __shared__ double s_c[MG_TILE + GS_HALO];
    __shared__ uint32_t s_head[MG_TILE + 1];
    __shared__ uint64_t s_scan[MG_THREADS / kWave];
    constexpr int MI = MG_TILE / MG_THREADS;
    static_assert(MI <= 4 && MG_TILE < 65536, "flags are packed 16 bits per round");
    const int64_t nb = (R + MG_TILE - 1) / MG_TILE;
    // monomial digits of a composite key, least significant (x_n) first
    auto to_fields = [&](uint64_t key) {
        uint64_t x = span ? key % span : key;
        uint64_t f = 0;
        for (int v = n - 1; v >= 0; --v) {
            const uint64_t q = x / radix;
            f |= (x - q * radix) << (bits * (n - 1 - v));
            x = q;
        }
        return f;
    };
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int64_t t0 = blk * MG_TILE;
        const int m = (int)(R - t0 < MG_TILE ? R - t0 : MG_TILE);
        const int hl = (int)(R - t0 - m < GS_HALO ? R - t0 - m : GS_HALO);
        __syncthreads();   // the previous tile's LDS reads are done
        uint64_t kr[MI + 1];
        double cr[MI + 1];
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * MG_THREADS + threadIdx.x;
            const int lc = l < m ? l : m - 1;
            kr[q] = keys[t0 + lc];
            cr[q] = coefs[vals[t0 + lc]];
        }
        kr[MI] = 0;
        cr[MI] = 0.0;
        if ((int)threadIdx.x < hl) {
            kr[MI] = keys[t0 + m + threadIdx.x];
            cr[MI] = coefs[vals[t0 + m + threadIdx.x]];
        }
        const uint64_t before = (threadIdx.x == 0 && t0 > 0) ? keys[t0 - 1] : 0ull;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * MG_THREADS + threadIdx.x;
            if (l < m) {
                s_key[l] = kr[q];
                s_c[l] = cr[q];
            }
        }
        if ((int)threadIdx.x < hl) {
            s_key[m + threadIdx.x] = kr[MI];
            s_c[m + threadIdx.x] = cr[MI];
        }
        __syncthreads();
        // ---- compact the run heads in element order
        uint64_t hflags = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * MG_THREADS + threadIdx.x;
            if (l < m) {
                const uint64_t key = s_key[l];
                const bool head = l > 0 ? s_key[l - 1] != key : (t0 == 0 || before != key);
                if (head) hflags |= 1ull << (16 * q);
            }
        }
        uint64_t htot;
        const uint64_t hpre = block_exclusive_scan<MG_THREADS>(hflags, s_scan, htot);
        int nh = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            if ((hflags >> (16 * q)) & 1u)
                s_head[nh + (int)((hpre >> (16 * q)) & 0xffffu)] = (uint32_t)(q * MG_THREADS + threadIdx.x);
            nh += (int)((htot >> (16 * q)) & 0xffffu);
        }
        if (threadIdx.x == 0) s_head[nh] = (uint32_t)m;
        __syncthreads();
        // ---- one run per lane
        uint64_t hk[MI];
        double hs[MI];
        uint64_t kflags = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int k = q * MG_THREADS + threadIdx.x;
            hk[q] = 0;
            hs[q] = 0.0;
            if (k < nh) {
                const int l = (int)s_head[k], e = (int)s_head[k + 1];
                const uint64_t key = s_key[l];
                double s = s_c[l];
                for (int f = l + 1; f < e; ++f) s = s + s_c[f];
                if (k == nh - 1) {
                    int f = m;
                    for (; f < m + hl && s_key[f] == key; ++f) s = s + s_c[f];
                    if (f == m + hl)
                        for (int64_t g = t0 + m + hl; g < R && keys[g] == key; ++g) s = s + coefs[vals[g]];
                }
                if (!(fabs(s) <= tol)) {
                    hk[q] = key;
                    hs[q] = s;
                    kflags |= 1ull << (16 * q);
                }
            }
        }
        uint64_t ktot;
        const uint64_t kpre = block_exclusive_scan<MG_THREADS>(kflags, s_scan, ktot);
        int64_t tot = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            if ((kflags >> (16 * q)) & 1u) {
                const int64_t d = t0 + tot + (int64_t)((kpre >> (16 * q)) & 0xffffu);
                st_key[d] = to_fields(hk[q]);
                st_ckey[d] = hk[q];
                st_coef[d] = hs[q];
            }
            tot += (int64_t)((ktot >> (16 * q)) & 0xffffu);
        }
        if (threadIdx.x == 0) {
            seg_count[blk] = tot;
            stage_off[blk] = t0;
        }
    }
}

// row_ptr[p] = number of kept terms whose key is below p * span: the first
// sorted element with such a key falls in merge tile b, every run staged by
// an earlier tile has a smaller key, and the staged keys of tile b are
// searched.  Threads p = 0..P; out_off holds nb + 1 entries (the last is the
// total).
__global__ void k_ws_rowptr(int64_t P, uint64_t span, const uint64_t *__restrict__ keys, int64_t R,
                            const int64_t *__restrict__ stage_off, const int64_t *__restrict__ seg_count,
                            const int64_t *__restrict__ out_off, int64_t nb, const uint64_t *__restrict__ st_ckey,
                            int64_t *row_ptr)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    if (p == 0) {
        row_ptr[0] = 0;
        return;
    }
    if (p == P) {
        row_ptr[P] = out_off[nb];
        return;
    }
    const uint64_t v = (uint64_t)p * span;   // 0 < p < P, so span > 0
    int64_t lo = 0, hi = R;                 // first element with key >= v
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    if (lo == R) {
        row_ptr[p] = out_off[nb];
        return;
    }
    const int64_t b = lo / MG_TILE;
    const uint64_t *sk = st_ckey + stage_off[b];
    int64_t a = 0, c = seg_count[b];
    while (a < c) {
        const int64_t mid = (a + c) >> 1;
        if (sk[mid] < v) a = mid + 1;
        else c = mid;
    }
    row_ptr[p] = out_off[b] + a;
}

}  // namespace polyhip
