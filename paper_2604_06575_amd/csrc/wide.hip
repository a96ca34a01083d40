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
//
// When p * r^n does not fit 64 bits (many variables, many polynomials), the
// key is cut into words at variable boundaries: word 0 holds the least
// significant variables, ..., the top word the polynomial index and the
// most significant variables, each a mixed-radix number below 2^64.  The LSD
// sort then runs word by word, least significant first: before a word's
// passes its keys are built in input order from the exponent rows
// (k_ww_word, coalesced) and gathered into the current order (k_ww_gather),
// so only the permutation travels between words.  Runs are found by comparing each element's top word and
// the exponents of the lower words with its predecessor's (k_ww_heads), the
// merge stages a representative term index per kept run (k_ww_merge), and
// the unpack copies that term's exponent row (k_ww_compact); the row
// pointers come from the top words as above.  The same path serves
// n * bit_width(max_exp) > 64, where exponents no longer fit one word of
// bit fields.
#include "kernels.h"

namespace polyhip {

namespace {

// The polynomial holding term t (the last p < P with row_ptr[p] <= t) for
// the consecutive terms t of one block: thread 0 binary-searches the block's
// first term t0, then each thread walks forward from there (a block of terms
// usually lies in one or two polynomials), instead of every thread walking
// a dependent chain of loads from the top.  Every thread of the block calls
// it; the result is meaningful for t < T only.
__device__ inline int64_t block_poly_of(const int64_t *__restrict__ row_ptr, int64_t P, int64_t t0, int64_t t,
                                        int64_t T)
{
    __shared__ int64_t s_a;
    if (threadIdx.x == 0) {
        int64_t a = 0, b = P;
        while (b - a > 1) {
            const int64_t mid = (a + b) >> 1;
            if (row_ptr[mid] <= t0) a = mid;
            else b = mid;
        }
        s_a = a;
    }
    __syncthreads();
    int64_t a = s_a;
    if (t < T)
        while (a + 1 < P && row_ptr[a + 1] <= t) ++a;
    return a;
}

}  // namespace

// span = r^n, or 0 for a single polynomial
__global__ void k_ws_keys(const uint8_t *__restrict__ exps, int64_t T, int n, uint32_t radix, int max_exp,
                          const int64_t *__restrict__ row_ptr, int64_t P, uint64_t span, uint64_t *__restrict__ keys,
                          uint32_t *__restrict__ vals, int32_t *status)
{
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x, t = t0 + threadIdx.x;
    const int64_t lo = block_poly_of(row_ptr, P, t0, t, T);   // the polynomial holding term t
    if (t >= T) return;
    const uint8_t *row = exps + t * n;
    uint64_t k = 0;
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t e = row[i];
        bad |= (int)(e > (uint32_t)max_exp);
        k = k * radix + e;
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

// keys[t] = the key word of variables [lo, hi) of term t, in input order:
// the mixed-radix number of those exponents, x_lo most significant, with
// the polynomial index above them (p * radix^(hi - lo)) when with_poly.
// Exponents above max_exp set POLY_ERR_EXPONENT (every variable is in
// exactly one word).
__global__ void k_ww_word(const uint8_t *__restrict__ exps, int64_t T, int n, uint32_t radix, int max_exp, int lo,
                          int hi, int with_poly, const int64_t *__restrict__ row_ptr, int64_t P,
                          uint64_t *__restrict__ keys, int32_t *status)
{
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x, t = t0 + threadIdx.x;
    uint64_t k = 0;
    if (with_poly) k = (uint64_t)block_poly_of(row_ptr, P, t0, t, T);
    if (t >= T) return;
    const uint8_t *row = exps + t * n;
    int bad = 0;
    if ((n & 3) == 0) {   // 4-byte aligned rows: one load per four exponents
        const uint32_t *row4 = reinterpret_cast<const uint32_t *>(row);
        uint32_t word = 0;
        int wi = -1;
        for (int v = lo; v < hi; ++v) {
            if ((v >> 2) != wi) {
                wi = v >> 2;
                word = row4[wi];
            }
            const uint32_t e = (word >> (8 * (v & 3))) & 0xffu;
            bad |= (int)(e > (uint32_t)max_exp);
            k = k * radix + e;
        }
    } else {
        for (int v = lo; v < hi; ++v) {
            const uint32_t e = row[v];
            bad |= (int)(e > (uint32_t)max_exp);
            k = k * radix + e;
        }
    }
    keys[t] = k;
    if (bad) set_status(status, POLY_ERR_EXPONENT);
}

// The two least significant words in one pass over the rows: keys0[t] for
// variables [lo0, hi0) and keys1[t] for [lo1, hi1) (with the polynomial
// index when with_poly); copy0, when given, receives keys0 again.
__global__ void k_ww_word2(const uint8_t *__restrict__ exps, int64_t T, int n, uint32_t radix, int max_exp,
                           int lo0, int hi0, int lo1, int hi1, int with_poly, const int64_t *__restrict__ row_ptr,
                           int64_t P, uint64_t *__restrict__ keys0, uint64_t *__restrict__ copy0,
                           uint64_t *__restrict__ keys1, int32_t *status)
{
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x, t = t0 + threadIdx.x;
    uint64_t k0 = 0, k1 = 0;
    if (with_poly) k1 = (uint64_t)block_poly_of(row_ptr, P, t0, t, T);
    if (t >= T) return;
    const uint8_t *row = exps + t * n;
    int bad = 0;
    // variables lo1 < hi1 <= lo0 < hi0: word 1 first, then word 0
    auto digits = [&](int lo, int hi, uint64_t &k) {
        if ((n & 3) == 0) {
            const uint32_t *row4 = reinterpret_cast<const uint32_t *>(row);
            uint32_t word = 0;
            int wi = -1;
            for (int v = lo; v < hi; ++v) {
                if ((v >> 2) != wi) {
                    wi = v >> 2;
                    word = row4[wi];
                }
                const uint32_t e = (word >> (8 * (v & 3))) & 0xffu;
                bad |= (int)(e > (uint32_t)max_exp);
                k = k * radix + e;
            }
        } else {
            for (int v = lo; v < hi; ++v) {
                const uint32_t e = row[v];
                bad |= (int)(e > (uint32_t)max_exp);
                k = k * radix + e;
            }
        }
    };
    digits(lo1, hi1, k1);
    digits(lo0, hi0, k0);
    keys0[t] = k0;
    if (copy0) copy0[t] = k0;
    keys1[t] = k1;
    if (bad) set_status(status, POLY_ERR_EXPONENT);
}

// head[i] for a two-word key: element i starts a run unless both its top
// and its low word equal element i - 1's.
__global__ void k_ww_heads2(const uint64_t *__restrict__ top, const uint64_t *__restrict__ low, int64_t R,
                            uint8_t *__restrict__ head)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R) return;
    head[i] = (uint8_t)(i == 0 || top[i] != top[i - 1] || low[i] != low[i - 1]);
}

// dst[i] = src[vals[i]]: a word's keys, built in input order, put in the
// current sorted order.
__global__ void k_ww_gather(const uint64_t *__restrict__ src, const uint32_t *__restrict__ vals, int64_t R,
                            uint64_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R) dst[i] = src[vals[i]];
}

// The identity permutation (before the first word's passes).
__global__ void k_ww_iota(uint32_t *vals, int64_t T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) vals[i] = (uint32_t)i;
}

// head[i] = 1 if sorted element i starts a run: its top word or its
// exponents of variables [lo, n) (those outside the top word) differ from
// element i - 1's.
__global__ void k_ww_heads(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t R,
                           const uint8_t *__restrict__ exps, int n, int lo, uint8_t *__restrict__ head)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R) return;
    bool h = i == 0 || keys[i] != keys[i - 1];
    if (!h) {
        const uint8_t *a = exps + (int64_t)vals[i] * n, *b = exps + (int64_t)vals[i - 1] * n;
        for (int v = lo; v < n; ++v) {
            if (a[v] != b[v]) {
                h = true;
                break;
            }
        }
    }
    head[i] = (uint8_t)h;
}

// As k_ws_merge, with the runs given by head flags: each run is summed left
// to right in one lane; a kept run stages its first element's term index
// (st_idx; for two-word keys the low word st_low instead), top word
// (st_ckey) and sum.
__global__ void __launch_bounds__(MG_THREADS) k_ww_merge(const uint64_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ vals,
                                                        const uint8_t *__restrict__ head, int64_t R,
                                                        const double *__restrict__ coefs, double tol,
                                                        uint32_t *__restrict__ st_idx, uint64_t *__restrict__ st_ckey,
                                                        double *__restrict__ st_coef, int64_t *seg_count,
                                                        int64_t *stage_off, const uint64_t *__restrict__ low,
                                                        uint64_t *__restrict__ st_low)
{
    __shared__ double s_c[MG_TILE + GS_HALO];
    __shared__ uint8_t s_h[MG_TILE + GS_HALO];
    __shared__ uint32_t s_head[MG_TILE + 1];
    __shared__ uint64_t s_scan[MG_THREADS / kWave];
    constexpr int MI = MG_TILE / MG_THREADS;
    static_assert(MI <= 4 && MG_TILE < 65536, "flags are packed 16 bits per round");
    const int64_t nb = (R + MG_TILE - 1) / MG_TILE;
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int64_t t0 = blk * MG_TILE;
        const int m = (int)(R - t0 < MG_TILE ? R - t0 : MG_TILE);
        const int hl = (int)(R - t0 - m < GS_HALO ? R - t0 - m : GS_HALO);
        __syncthreads();   // the previous tile's LDS reads are done
        for (int l = threadIdx.x; l < m + hl; l += MG_THREADS) {
            s_c[l] = coefs[vals[t0 + l]];
            s_h[l] = head[t0 + l];
        }
        __syncthreads();
        uint64_t hflags = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * MG_THREADS + threadIdx.x;
            if (l < m && s_h[l]) hflags |= 1ull << (16 * q);
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
        int hl_k[MI];
        double hs[MI];
        uint64_t kflags = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int k = q * MG_THREADS + threadIdx.x;
            hl_k[q] = 0;
            hs[q] = 0.0;
            if (k < nh) {
                const int l = (int)s_head[k], e = (int)s_head[k + 1];
                double s = s_c[l];
                for (int f = l + 1; f < e; ++f) s = s + s_c[f];
                if (k == nh - 1) {
                    int f = m;
                    for (; f < m + hl && !s_h[f]; ++f) s = s + s_c[f];
                    if (f == m + hl)
                        for (int64_t g = t0 + m + hl; g < R && !head[g]; ++g) s = s + coefs[vals[g]];
                }
                if (!(fabs(s) <= tol)) {
                    hl_k[q] = l;
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
                st_ckey[d] = keys[t0 + hl_k[q]];
                st_coef[d] = hs[q];
                if (low) st_low[d] = low[t0 + hl_k[q]];
                else st_idx[d] = vals[t0 + hl_k[q]];
            }
            tot += (int64_t)((ktot >> (16 * q)) & 0xffffu);
        }
        if (threadIdx.x == 0) {
            seg_count[blk] = tot;
            stage_off[blk] = t0;
        }
    }
}

// Raw product sizes of the pairs a_p * b_p.
__global__ void k_mul_raw_sizes(const int64_t *a_rp, const int64_t *b_rp, int64_t P, int64_t *sizes)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) sizes[p] = (a_rp[p + 1] - a_rp[p]) * (b_rp[p + 1] - b_rp[p]);
}

// The raw products of the pairs as exponent rows and coefficients, in the
// order of the definition (pair by pair, term i of a_p then term j of b_p,
// i-major): element k of pair p is (i, j) = divmod(k - r_rp[p], |b_p|), row
// a_i + b_j, coefficient fl(c_i * c_j).  One thread per raw term.
__global__ void k_mul_expand_rows(const int64_t *__restrict__ a_rp, const uint8_t *__restrict__ a_e,
                                  const double *__restrict__ a_c, int a_max, const int64_t *__restrict__ b_rp,
                                  const uint8_t *__restrict__ b_e, const double *__restrict__ b_c, int b_max,
                                  int64_t P, int n, const int64_t *__restrict__ r_rp, int64_t R,
                                  uint8_t *__restrict__ r_e, double *__restrict__ r_c, int32_t *status)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= R) return;
    int64_t lo = 0, hi = P;   // the last p with r_rp[p] <= k
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (r_rp[mid] <= k) lo = mid;
        else hi = mid;
    }
    const int64_t nb = b_rp[lo + 1] - b_rp[lo];
    const int64_t l = k - r_rp[lo], i = l / nb, j = l - i * nb;
    const int64_t ia = a_rp[lo] + i, jb = b_rp[lo] + j;
    const uint8_t *ra = a_e + ia * n, *rb = b_e + jb * n;
    uint8_t *o = r_e + k * n;
    int bad = 0;
    for (int v = 0; v < n; ++v) {
        const uint32_t x = ra[v], y = rb[v];
        bad |= (int)(x > (uint32_t)a_max) | (int)(y > (uint32_t)b_max);
        o[v] = (uint8_t)(x + y);
    }
    r_c[k] = a_c[ia] * b_c[jb];
    if (bad) set_status(status, POLY_ERR_EXPONENT);
}

// Unpack of the staged runs of merge tile blockIdx.x: coefficients, and each
// run's exponent row copied from its representative input term.  Block
// (b, y) takes rows y * 256 .. y * 256 + 255 of the tile, 64 per wave; a
// wave copies its rows' bytes as one contiguous output run, lane by lane
// (4-byte words when rows are 4-byte aligned), so the stores are coalesced
// and the loads of one row come from one instruction.
__global__ void __launch_bounds__(256) k_ww_compact(const int64_t *__restrict__ stage_off,
                                                    const int64_t *__restrict__ seg_count,
                                                    const int64_t *__restrict__ out_off,
                                                    const uint32_t *__restrict__ st_idx,
                                                    const double *__restrict__ st_coef,
                                                    const uint8_t *__restrict__ exps, int n,
                                                    uint8_t *__restrict__ out_exps, double *__restrict__ out_coefs,
                                                    int64_t capacity, int32_t *status)
{
    const int64_t b = blockIdx.x;
    const int64_t cnt = seg_count[b], src = stage_off[b], dst = out_off[b];
    if (threadIdx.x == 0 && blockIdx.y == 0 && dst + cnt > capacity) set_status(status, POLY_ERR_CAPACITY);
    const int64_t end = dst + cnt < capacity ? dst + cnt : capacity;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t r0 = dst + (int64_t)blockIdx.y * blockDim.x + (int64_t)wave * kWave;
    if (r0 >= end) return;
    const int rows = (int)(end - r0 < kWave ? end - r0 : kWave);
    uint32_t my_idx = 0;
    if (lane < rows) {
        out_coefs[r0 + lane] = st_coef[src + (r0 - dst) + lane];
        my_idx = st_idx[src + (r0 - dst) + lane];
    }
    if ((n & 3) == 0) {
        const uint32_t nw = (uint32_t)n / 4;
        const uint32_t *ex4 = reinterpret_cast<const uint32_t *>(exps);
        uint32_t *out4 = reinterpret_cast<uint32_t *>(out_exps) + r0 * nw;
        const uint32_t total = (uint32_t)rows * nw;
        // uniform trip count: every lane takes part in each shuffle
        for (uint32_t d0 = 0; d0 < total; d0 += kWave) {
            const uint32_t d = d0 + lane;
            const uint32_t r = d / nw, w = d - r * nw;
            const uint32_t t = (uint32_t)__shfl((int)my_idx, (int)(r < kWave ? r : kWave - 1), kWave);
            if (d < total) out4[d] = ex4[(int64_t)t * nw + w];
        }
    } else {
        const uint32_t un = (uint32_t)n;
        uint8_t *out = out_exps + r0 * n;
        const uint32_t total = (uint32_t)rows * un;
        for (uint32_t d0 = 0; d0 < total; d0 += kWave) {
            const uint32_t d = d0 + lane;
            const uint32_t r = d / un, c = d - r * un;
            const uint32_t t = (uint32_t)__shfl((int)my_idx, (int)(r < kWave ? r : kWave - 1), kWave);
            if (d < total) out[d] = exps[(int64_t)t * n + c];
        }
    }
}

// Unpack of the staged runs of merge tile blockIdx.x for a two-word key:
// the exponents are the mixed-radix digits of the top word (variables
// [0, split), the polynomial index above them) and of the low word
// (variables [split, n)), peeled least significant first by multiply-high
// divisions (each quotient from floor((2^w - 1) / divisor) is exact or one
// short, then corrected).  Each thread writes its row into the wave's LDS buffer; the
// wave then stores its 64 rows as one contiguous run (4-byte words when
// rows are 4-byte aligned).  Block (b, y) takes rows y * 256 .. + 255 of
// the tile.  Dynamic LDS: 256 * n bytes.
__global__ void __launch_bounds__(256) k_ww_compact2(const int64_t *__restrict__ stage_off,
                                                     const int64_t *__restrict__ seg_count,
                                                     const int64_t *__restrict__ out_off,
                                                     const uint64_t *__restrict__ st_top,
                                                     const uint64_t *__restrict__ st_low,
                                                     const double *__restrict__ st_coef, int n, int split,
                                                     uint64_t radix, int chunk, uint64_t div, uint64_t div_magic,
                                                     uint32_t digit_magic, uint8_t *__restrict__ out_exps,
                                                     double *__restrict__ out_coefs, int64_t capacity,
                                                     int32_t *status)
{
    extern __shared__ uint8_t s_rows[];
    const int64_t b = blockIdx.x;
    const int64_t cnt = seg_count[b], src = stage_off[b], dst = out_off[b];
    if (threadIdx.x == 0 && blockIdx.y == 0 && dst + cnt > capacity) set_status(status, POLY_ERR_CAPACITY);
    const int64_t end = dst + cnt < capacity ? dst + cnt : capacity;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t r0 = dst + (int64_t)blockIdx.y * blockDim.x + (int64_t)wave * kWave;
    if (r0 >= end) return;
    const int rows = (int)(end - r0 < kWave ? end - r0 : kWave);
    uint8_t *buf = s_rows + (size_t)wave * kWave * n;
    // digits least significant first: a chunk of `chunk` digits (radix^chunk
    // below 2^32) is split off with one 64-bit multiply-high division by
    // div = radix^chunk, then its digits with 32-bit ones.  The last chunk is
    // split off too: the top word holds the polynomial index above its digits.
    const uint32_t r32 = (uint32_t)radix;
    auto digits = [&](uint64_t x, int v_hi, int v_lo, uint8_t *row) {
        int v = v_hi - 1;
        while (v >= v_lo) {
            uint64_t q = __umul64hi(x, div_magic);
            uint64_t rem = x - q * div;
            if (rem >= div) {
                ++q;
                rem -= div;
            }
            uint32_t part = (uint32_t)rem;
            x = q;
            const int e = v - v_lo + 1 < chunk ? v - v_lo + 1 : chunk;
            for (int j = 0; j < e; ++j, --v) {
                uint32_t dq = __umulhi(part, digit_magic);
                uint32_t dr = part - dq * r32;
                if (dr >= r32) {
                    ++dq;
                    dr -= r32;
                }
                row[v] = (uint8_t)dr;
                part = dq;
            }
        }
    };
    if (lane < rows) {
        const int64_t k = src + (r0 - dst) + lane;
        out_coefs[r0 + lane] = st_coef[k];
        uint8_t *row = buf + lane * n;
        digits(st_low[k], n, split, row);
        digits(st_top[k], split, 0, row);   // the polynomial index above them is left over
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t total = (uint32_t)rows * (uint32_t)n;
    if ((n & 3) == 0) {
        const uint32_t *b4 = reinterpret_cast<const uint32_t *>(buf);
        uint32_t *o4 = reinterpret_cast<uint32_t *>(out_exps + r0 * n);
        for (uint32_t d = lane; d < total / 4; d += kWave) o4[d] = b4[d];
    } else {
        uint8_t *o = out_exps + r0 * n;
        for (uint32_t d = lane; d < total; d += kWave) o[d] = buf[d];
    }
}

}  // namespace polyhip
