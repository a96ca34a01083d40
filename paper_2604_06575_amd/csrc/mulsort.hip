// times + simplify of one large pair by a global stable radix sort
// (Section 3.3 entrywise `times`, Table "coresemantics" simplify).
//
// The raw product of p (ta terms) and q (tb terms) is generated in (i, j)
// order -- i over p's terms in storage order, j over q's terms in ascending
// key order (a stable order, so equal keys of q keep storage order) -- as
// (packed key k_i + k_j, raw index i * tb + j).  A least-significant-digit
// radix sort with GS_BITS-bit digits, stable in every pass, orders the pairs
// by key while keeping (i, j) order among equal keys.  Each run of equal keys
// is then summed left to right by one lane, with every product c_i * c_j
// recomputed from the raw index, so the sums are the sequential ones of the
// definition; runs with |s| <= tol are dropped and the rest staged for the
// shared unpack kernel.  All traffic is streaming HBM traffic: the sort is
// bandwidth-bound, with no per-row state on chip.
#include "kernels.h"
#include "lds_sort.h"

// products and sums are rounded separately, as in the definition (no FMA)
#pragma clang fp contract(off)

namespace polyhip {

// The partner operand in ascending key order, stably (equal keys keep
// storage order), in one workgroup (T <= GS_SORT1_CAP): sorted keys, the
// storage index of each sorted position, and the coefficients in sorted
// order.  Keys are sorted relative to their minimum, on the occupied bits.
// Dynamic LDS: GS_SORT1_CAP * 12 bytes.
__global__ void __launch_bounds__(GS_THREADS) k_gs_sort_partner(const uint64_t *keys, const double *coefs, int64_t T,
                                                               uint64_t *keys_s, uint32_t *perm, double *coefs_s)
{
    extern __shared__ uint64_t s_dyn[];
    uint64_t *sk = s_dyn;
    uint32_t *sv = reinterpret_cast<uint32_t *>(s_dyn + GS_SORT1_CAP);
    __shared__ uint32_t s_cnt[(GS_THREADS / kWave) * 256];
    __shared__ uint32_t s_scan[GS_THREADS / kWave];
    __shared__ uint64_t s_red[GS_THREADS / kWave];
    const int m = (int)T;
    uint64_t lmin = ~0ull, lmax = 0;
    for (int i = threadIdx.x; i < m; i += GS_THREADS) {
        const uint64_t k = keys[i];
        sk[i] = k;
        sv[i] = (uint32_t)i;
        lmin = k < lmin ? k : lmin;
        lmax = k > lmax ? k : lmax;
    }
    const uint64_t kmin = block_min_u64<GS_THREADS>(lmin, s_red);
    const uint64_t kmax = block_max_u64<GS_THREADS>(lmax, s_red);
    for (int i = threadIdx.x; i < m; i += GS_THREADS) sk[i] -= kmin;
    __syncthreads();
    const int bits = kmax > kmin ? 64 - __clzll((unsigned long long)(kmax - kmin)) : 0;
    lds_radix_sort<GS_THREADS, GS_SORT1_CAP / GS_THREADS, uint32_t>(sk, sv, m, bits, s_cnt, s_scan);
    for (int i = threadIdx.x; i < m; i += GS_THREADS) {
        keys_s[i] = sk[i] + kmin;
        perm[i] = sv[i];
        coefs_s[i] = coefs[sv[i]];
    }
}

// raw pair (i, j) -> (key, i * tb + j), one block row per term of p
__global__ void __launch_bounds__(GS_THREADS) k_gs_generate(const uint64_t *ka, const uint64_t *kb_s, int64_t ta,
                                                           int64_t tb, uint64_t *keys, uint32_t *vals)
{
    for (int64_t i = blockIdx.x; i < ta; i += gridDim.x) {
        const uint64_t kr = ka[i];
        const int64_t base = i * tb;
        for (int64_t j = threadIdx.x; j < tb; j += GS_THREADS) {
            keys[base + j] = kr + kb_s[j];
            vals[base + j] = (uint32_t)(base + j);
        }
    }
}

// Per-tile digit counts, digit-major: hist[d * nblocks + b].  One wave
// counts a whole tile into its own LDS histogram, with no barrier: lanes
// holding the same digit are found with wavefront ballots and their lowest
// lane adds the group size.  Waves take tiles wave_id, wave_id + total
// waves, ... (few, long-lived workgroups rather than one per tile).
__global__ void __launch_bounds__(GS_HIST_THREADS) k_gs_hist(const uint64_t *keys, int64_t R, int shift,
                                                            int64_t nblocks, int64_t *hist)
{
    constexpr int W = GS_HIST_THREADS / kWave;
    constexpr int UN = 8;   // key loads in flight per lane
    __shared__ uint32_t s_cnt[W][GS_BINS];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const unsigned long long lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    uint32_t *cnt = s_cnt[w];
    const int64_t nwaves = (int64_t)gridDim.x * W;
    for (int64_t tile = (int64_t)blockIdx.x * W + w; tile < nblocks; tile += nwaves) {
        for (int d = lane; d < GS_BINS; d += kWave) cnt[d] = 0;
        const int64_t t0 = tile * GS_TILE;
        const int m = (int)(R - t0 < GS_TILE ? R - t0 : GS_TILE);
        for (int c0 = 0; c0 < m; c0 += UN * kWave) {
            uint32_t dg[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int l = c0 + u * kWave + lane;
                dg[u] = l < m ? (uint32_t)(keys[t0 + l] >> shift) & (GS_BINS - 1) : (uint32_t)GS_BINS;
            }
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const uint32_t d = dg[u];
                unsigned long long peer = __ballot(d < (uint32_t)GS_BINS);   // padding lanes are in no group
#pragma unroll
                for (int bit = 0; bit < GS_BITS; ++bit) {
                    const bool set = (d >> bit) & 1u;
                    const unsigned long long bb = __ballot(set);
                    peer &= set ? bb : ~bb;
                }
                if (d < (uint32_t)GS_BINS && (peer & lt) == 0) cnt[d] += (uint32_t)__popcll(peer);
            }
        }
        for (int d = lane; d < GS_BINS; d += kWave) hist[(int64_t)d * nblocks + tile] = cnt[d];
    }
}

// One stable pass: the tile is ranked by digit in LDS (wavefront ballots,
// element order (wave, item, lane)), reordered in LDS, and written out so
// that each digit's elements leave as one contiguous run at
// hist_off[d * nblocks + b].
__global__ void __launch_bounds__(GS_THREADS) k_gs_scatter(const uint64_t *keys_in, const uint32_t *vals_in,
                                                          int64_t R, int shift, int64_t nblocks,
                                                          const int64_t *hist_off, uint64_t *keys_out,
                                                          uint32_t *vals_out)
{
    constexpr int W = GS_THREADS / kWave;
    __shared__ uint64_t s_key[GS_TILE];
    __shared__ uint32_t s_val[GS_TILE];
    __shared__ uint32_t s_cnt[W][GS_BINS];
    __shared__ uint32_t s_tot[GS_BINS];
    __shared__ uint32_t s_start[GS_BINS];
    __shared__ uint32_t s_scan[W];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const unsigned long long lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    const int64_t t0 = (int64_t)blockIdx.x * GS_TILE;
    const int m = (int)(R - t0 < GS_TILE ? R - t0 : GS_TILE);
    uint64_t k[GS_ITEMS];
    uint32_t v[GS_ITEMS], dg[GS_ITEMS], rank[GS_ITEMS];
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const int e = (w * GS_ITEMS + it) * kWave + lane;
        const bool valid = e < m;
        k[it] = valid ? keys_in[t0 + e] : ~0ull;   // padding sorts after every valid element
        v[it] = valid ? vals_in[t0 + e] : 0u;
        dg[it] = valid ? (uint32_t)(k[it] >> shift) & (GS_BINS - 1) : (uint32_t)(GS_BINS - 1);
    }
    for (int i = threadIdx.x; i < W * GS_BINS; i += GS_THREADS) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const uint32_t d = dg[it];
        unsigned long long peer = ~0ull;
#pragma unroll
        for (int bit = 0; bit < GS_BITS; ++bit) {
            const bool set = (d >> bit) & 1u;
            const unsigned long long bb = __ballot(set);
            peer &= set ? bb : ~bb;
        }
        const uint32_t prior = s_cnt[w][d];
        rank[it] = prior + (uint32_t)__popcll(peer & lt);
        if ((peer & lt) == 0) s_cnt[w][d] = prior + (uint32_t)__popcll(peer);   // lowest lane of the group
    }
    __syncthreads();
    // wave prefixes per digit (in place) and digit totals of the tile
    for (int d = threadIdx.x; d < GS_BINS; d += GS_THREADS) {
        uint32_t run = 0;
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = s_cnt[ww][d];
            s_cnt[ww][d] = run;
            run += c;
        }
        s_tot[d] = run;
    }
    __syncthreads();
    {
        uint32_t tot;
        const uint32_t x = threadIdx.x < GS_BINS ? s_tot[threadIdx.x] : 0u;
        const uint32_t ex = block_exclusive_scan<GS_THREADS>(x, s_scan, tot);
        if (threadIdx.x < GS_BINS) s_start[threadIdx.x] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const uint32_t d = dg[it];
        const uint32_t lp = s_start[d] + s_cnt[w][d] + rank[it];
        s_key[lp] = k[it];
        s_val[lp] = v[it];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < m; l += GS_THREADS) {
        const uint64_t key = s_key[l];
        const uint32_t d = (uint32_t)(key >> shift) & (GS_BINS - 1);
        const int64_t gpos = hist_off[(int64_t)d * nblocks + blockIdx.x] + (l - (int64_t)s_start[d]);
        keys_out[gpos] = key;
        vals_out[gpos] = s_val[l];
    }
}

// Runs of equal keys in the sorted stream.  Per tile of GS_TILE elements:
// the keys are staged in LDS and every lane forms the products c_i * c_j of
// its elements from the raw indices, (i, j) = (r / tb, r % tb), into LDS, so
// all coefficient gathers are in flight at once; the run heads (first
// elements of runs) are compacted in element order, and lane k then sums
// run k left to right from LDS -- one run per lane, so every lane has work
// -- continuing from global memory when the tile's last run runs past the
// tile.  Kept sums are staged in element order at [b * GS_TILE, ...).
// Persistent workgroups take tiles b = blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ void __launch_bounds__(GS_THREADS) k_gs_merge(const uint64_t *keys, const uint32_t *vals, int64_t R,
                                                        int64_t ta, int64_t tb, const double *ca,
                                                        const double *cb_s, double tol, uint64_t *st_key,
                                                        double *st_coef, int64_t *seg_count, int64_t *stage_off)
{
    __shared__ uint64_t s_key[GS_TILE];
    __shared__ double s_prod[GS_TILE];
    __shared__ uint32_t s_head[GS_TILE + 1];
    __shared__ uint64_t s_scan[GS_THREADS / kWave];
    constexpr int MI = GS_TILE / GS_THREADS;
    static_assert(MI <= 4 && GS_THREADS < 65536, "flags are packed 16 bits per round");
    (void)ta;
    const int64_t nb = (R + GS_TILE - 1) / GS_TILE;
    const uint32_t tb32 = (uint32_t)tb;
    const double inv_tb = 1.0 / (double)tb;
    auto product = [&](uint32_t r) {
        // r / tb in double precision (within one of the quotient for 32-bit r), then corrected
        uint32_t i = (uint32_t)((double)r * inv_tb);
        if (i * (uint64_t)tb32 > r) --i;
        else if ((uint64_t)(i + 1) * tb32 <= r) ++i;
        const uint32_t j = r - i * tb32;
        return ca[i] * cb_s[j];
    };
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int64_t t0 = blk * GS_TILE;
        const int m = (int)(R - t0 < GS_TILE ? R - t0 : GS_TILE);
        __syncthreads();   // the previous tile's LDS reads are done
        uint32_t vr[MI];
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * GS_THREADS + threadIdx.x;
            if (l < m) {
                s_key[l] = keys[t0 + l];
                vr[q] = vals[t0 + l];
            }
        }
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * GS_THREADS + threadIdx.x;
            if (l < m) s_prod[l] = product(vr[q]);
        }
        const uint64_t before = t0 > 0 ? keys[t0 - 1] : 0ull;
        __syncthreads();
        // ---- compact the run heads in element order
        uint64_t hflags = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * GS_THREADS + threadIdx.x;
            if (l < m) {
                const uint64_t key = s_key[l];
                const bool head = l > 0 ? s_key[l - 1] != key : (t0 == 0 || before != key);
                if (head) hflags |= 1ull << (16 * q);
            }
        }
        uint64_t htot;
        const uint64_t hpre = block_exclusive_scan<GS_THREADS>(hflags, s_scan, htot);
        int nh = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            if ((hflags >> (16 * q)) & 1u)
                s_head[nh + (int)((hpre >> (16 * q)) & 0xffffu)] = (uint32_t)(q * GS_THREADS + threadIdx.x);
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
            const int k = q * GS_THREADS + threadIdx.x;
            hk[q] = 0;
            hs[q] = 0.0;
            if (k < nh) {
                const int l = (int)s_head[k], e = (int)s_head[k + 1];
                const uint64_t key = s_key[l];
                double s = s_prod[l];
                for (int f = l + 1; f < e; ++f) s = s + s_prod[f];
                if (k == nh - 1)
                    for (int64_t g = t0 + m; g < R && keys[g] == key; ++g) s = s + product(vals[g]);
                if (!(fabs(s) <= tol)) {
                    hk[q] = key;
                    hs[q] = s;
                    kflags |= 1ull << (16 * q);
                }
            }
        }
        uint64_t ktot;
        const uint64_t kpre = block_exclusive_scan<GS_THREADS>(kflags, s_scan, ktot);
        int64_t tot = 0;
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            if ((kflags >> (16 * q)) & 1u) {
                const int64_t d = t0 + tot + (int64_t)((kpre >> (16 * q)) & 0xffffu);
                st_key[d] = hk[q];
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

// row_ptr of the single output polynomial: [0, total]
__global__ void k_gs_rowptr(const int64_t *out_off, int64_t nblocks, int64_t *row_ptr)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        row_ptr[0] = 0;
        row_ptr[1] = out_off[nblocks];
    }
}

}  // namespace polyhip
