// times + simplify of one large pair by a global stable radix sort
// (Section 3.3 entrywise `times`, Table "coresemantics" simplify).
//
// Keys here are mixed-radix numbers: with radix r = max_exp(p) + max_exp(q)
// + 1, the row e has key sum_i e_i r^(n-1-i), x1 most significant.  The key
// order is the lexicographic order of exponent rows, and since every
// exponent of a product is below r, a product key is the plain sum of its
// factors' keys.  The range r^n is usually far below that of bit fields
// (r rounded up to a power of two), so fewer digits need sorting.
//
// The raw product of p (ta terms) and q (tb terms) is generated in (i, j)
// order -- both operands in storage order, the order of the definition -- as
// (key k_i + k_j, raw index i * tb + j).  A least-significant-digit radix
// sort with digits of at most "sort_digit_bits" bits (a tunable; as few
// passes as the key range needs, digits as even as possible), stable in every pass, orders the pairs
// by key while keeping (i, j) order among equal keys.  Each run of equal keys
// is then summed left to right by one lane, with every product c_i * c_j
// recomputed from the raw index, so the sums are the sequential ones of the
// definition; runs with |s| <= tol are dropped and the rest staged for the
// shared unpack kernel.  All traffic is streaming HBM traffic: the sort is
// bandwidth-bound, with no per-row state on chip.
#include "kernels.h"

// products and sums are rounded separately, as in the definition (no FMA)
#pragma clang fp contract(off)

namespace polyhip {

// Mixed-radix key of each exponent row (Horner's rule, x1 first); rows with
// an exponent above max_exp set POLY_ERR_EXPONENT.
__global__ void k_gs_pack_radix(const uint8_t *exps, int64_t T, int n, uint64_t radix, int max_exp,
                                uint64_t *keys, int32_t *status)
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
    keys[t] = k;
    if (bad) set_status(status, POLY_ERR_EXPONENT);
}

// raw pair (i, j) -> (key, i * tb + j), one block row per term of p
__global__ void __launch_bounds__(GS_THREADS) k_gs_generate(const uint64_t *ka, const uint64_t *kb, int64_t ta,
                                                           int64_t tb, uint64_t *keys, uint32_t *vals)
{
    for (int64_t i = blockIdx.x; i < ta; i += gridDim.x) {
        const uint64_t kr = ka[i];
        const int64_t base = i * tb;
        for (int64_t j = threadIdx.x; j < tb; j += GS_THREADS) {
            keys[base + j] = kr + kb[j];
            vals[base + j] = (uint32_t)(base + j);
        }
    }
}

// Per-tile digit counts, digit-major: hist[d * nblocks + b].  One wave
// counts a whole tile into its own LDS histogram, with no barrier: every
// lane adds its element by an LDS atomic (lanes of one digit are serialized
// by the hardware; grouping them with wavefront ballots first cost more
// issue slots than it saved).  Waves take tiles wave_id, wave_id + total
// waves, ... (few, long-lived workgroups rather than one per tile).
template <int DB, bool GEN>
__global__ void __launch_bounds__(GS_HIST_THREADS) k_gs_hist(const uint64_t *keys, int64_t R, int shift,
                                                            int64_t nblocks, int64_t *hist, GsGen gen)
{
    constexpr int W = GS_HIST_THREADS / kWave;
    constexpr int UN = 8;   // key loads in flight per lane
    constexpr int NB = 1 << DB;
    __shared__ uint32_t s_cnt[W][NB];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    uint32_t *cnt = s_cnt[w];
    const int64_t nwaves = (int64_t)gridDim.x * W;
    for (int64_t tile = (int64_t)blockIdx.x * W + w; tile < nblocks; tile += nwaves) {
        for (int d = lane; d < NB; d += kWave) cnt[d] = 0;
        const int64_t t0 = tile * GS_TILE;
        const int m = (int)(R - t0 < GS_TILE ? R - t0 : GS_TILE);
        GsGen::Cursor cur;
        for (int c0 = 0; c0 < m; c0 += UN * kWave) {
            // loads unconditional (index clamped into the tile) so all UN are in
            // flight together; lanes past the tile get the padding digit
            uint64_t kv[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int l = c0 + u * kWave + lane;
                const int64_t g = t0 + (l < m ? l : m - 1);
                if (GEN) kv[u] = (c0 == 0 && u == 0) ? gen.first((uint32_t)g, cur) : gen.next((uint32_t)g, cur);
                else kv[u] = keys[g];
            }
            uint32_t dg[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int l = c0 + u * kWave + lane;
                dg[u] = l < m ? (uint32_t)(kv[u] >> shift) & (NB - 1) : (uint32_t)NB;
            }
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (dg[u] < (uint32_t)NB) atomicAdd(&cnt[dg[u]], 1u);   // padding lanes add nothing
        }
        for (int d = lane; d < NB; d += kWave) hist[(int64_t)d * nblocks + tile] = cnt[d];
    }
}

// One stable pass: the tile is ranked by digit in LDS (wavefront ballots,
// element order (wave, item, lane)), reordered in LDS, and written out so
// that each digit's elements leave as one contiguous run at
// hist_off[d * nblocks + b].
//
// Block 0 also zeroes `clear` (clear_n words): the state of the scan that
// produced hist_off, ready for the next pass.
//
// MODE selects the element format: GS_KV (key array + raw index array, in
// and out), GS_GEN_KV / GS_GEN_TO_PACKED (the first pass: elements generated
// from the operands, out as GS_KV / as GS_KV_TO_PACKED), GS_KV_TO_PACKED
// (key + raw index in; out one word per element,
// (key >> DB) << raw_bits | raw index: the digits still to sort above the
// raw index -- the first pass of a sort whose remaining digits and raw index
// fit 64 bits), GS_PACKED (packed words in and out).
template <int DB, int MODE>
__global__ void __launch_bounds__(GS_SC_THREADS) k_gs_scatter(const uint64_t *keys_in, const uint32_t *vals_in,
                                                          int64_t R, int shift, int64_t nblocks,
                                                          const int64_t *hist_off, uint64_t *keys_out,
                                                          uint32_t *vals_out, int raw_bits,
                                                          unsigned long long *clear, int64_t clear_n, GsGen gen)
{
    // the scan that produced hist_off is done: reset its state for the next one
    if (blockIdx.x == 0)
        for (int64_t i = threadIdx.x; i < clear_n; i += GS_SC_THREADS) clear[i] = 0ull;
    constexpr int W = GS_SC_THREADS / kWave;
    constexpr int NB = 1 << DB;
    constexpr bool HAS_VALS = MODE != GS_PACKED;
    constexpr bool GEN = MODE == GS_GEN_KV || MODE == GS_GEN_TO_PACKED;
    __shared__ uint64_t s_key[GS_TILE];
    // raw indices staged beside the keys; generated ones are t0 + (offset in
    // the tile), so 16 bits each (LDS for three workgroups per CU, not two)
    __shared__ uint32_t s_val[HAS_VALS && !GEN ? GS_TILE : 1];
    __shared__ uint16_t s_gen[GEN ? GS_TILE : 1];
    __shared__ uint32_t s_cnt[W][NB];
    __shared__ uint32_t s_tot[NB];
    __shared__ uint32_t s_start[NB];
    __shared__ uint32_t s_scan[W];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const unsigned long long lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    const int64_t t0 = (int64_t)blockIdx.x * GS_TILE;
    const int m = (int)(R - t0 < GS_TILE ? R - t0 : GS_TILE);
    uint64_t k[GS_ITEMS];
    uint32_t v[GS_ITEMS], dg[GS_ITEMS], rank[GS_ITEMS];
    // loads unconditional (index clamped into the tile) so all are in flight together
    GsGen::Cursor cur;
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const int e = (w * GS_ITEMS + it) * kWave + lane;
        const int ec = e < m ? e : m - 1;
        if (GEN) {
            v[it] = (uint32_t)(t0 + ec);
            k[it] = it == 0 ? gen.first(v[it], cur) : gen.next(v[it], cur);
        } else {
            k[it] = keys_in[t0 + ec];
            v[it] = HAS_VALS ? vals_in[t0 + ec] : 0u;
        }
    }
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const int e = (w * GS_ITEMS + it) * kWave + lane;
        const bool valid = e < m;
        k[it] = valid ? k[it] : ~0ull;   // padding sorts after every valid element
        dg[it] = valid ? (uint32_t)(k[it] >> shift) & (NB - 1) : (uint32_t)(NB - 1);
    }
    for (int i = threadIdx.x; i < W * NB; i += GS_SC_THREADS) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const uint32_t d = dg[it];
        unsigned long long peer = ~0ull;
#pragma unroll
        for (int bit = 0; bit < DB; ++bit) {
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
    for (int d = threadIdx.x; d < NB; d += GS_SC_THREADS) {
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
        // digit starts: each thread scans PER consecutive digits
        constexpr int PER = (NB + GS_SC_THREADS - 1) / GS_SC_THREADS;
        uint32_t loc[PER], sum = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int d = threadIdx.x * PER + i;
            loc[i] = d < NB ? s_tot[d] : 0u;
            sum += loc[i];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<GS_SC_THREADS>(sum, s_scan, tot);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int d = threadIdx.x * PER + i;
            if (d < NB) s_start[d] = ex;
            ex += loc[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < GS_ITEMS; ++it) {
        const uint32_t d = dg[it];
        const uint32_t lp = s_start[d] + s_cnt[w][d] + rank[it];
        s_key[lp] = k[it];
        if (GEN) s_gen[lp] = (uint16_t)(v[it] - (uint32_t)t0);
        else if (HAS_VALS) s_val[lp] = v[it];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < m; l += GS_SC_THREADS) {
        const uint64_t key = s_key[l];
        const uint32_t d = (uint32_t)(key >> shift) & (NB - 1);
        const int64_t gpos = hist_off[(int64_t)d * nblocks + blockIdx.x] + (l - (int64_t)s_start[d]);
        const uint32_t val = GEN ? (uint32_t)t0 + s_gen[l] : (HAS_VALS ? s_val[l] : 0u);
        if (MODE == GS_KV || MODE == GS_GEN_KV) {
            keys_out[gpos] = key;
            vals_out[gpos] = val;
        } else if (MODE == GS_KV_TO_PACKED || MODE == GS_GEN_TO_PACKED) {
            keys_out[gpos] = ((key >> DB) << raw_bits) | (uint64_t)val;
        } else {
            keys_out[gpos] = key;
        }
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
//
// PACKED: the sorted stream holds packed words (raw index in the low
// raw_bits bits, `vals` unused); each element's key is rebuilt exactly as
// ka[i] + kb[j] from its raw index.
template <bool PACKED>
__global__ void __launch_bounds__(MG_THREADS) k_gs_merge(const uint64_t *keys, const uint32_t *vals, int64_t R,
                                                        int64_t ta, int64_t tb, const uint64_t *ka,
                                                        const uint64_t *kb, int raw_bits, const double *ca,
                                                        const double *cb, const GsKC *pa, const GsKC *pb,
                                                        double tol, RadixDecode dec, uint64_t *st_key,
                                                        double *st_coef, int64_t *seg_count, int64_t *stage_off)
{
    __shared__ uint64_t s_key[MG_TILE + GS_HALO];
    __shared__ double s_prod[MG_TILE + GS_HALO];
    __shared__ uint32_t s_head[MG_TILE + 1];
    __shared__ uint64_t s_scan[MG_THREADS / kWave];
    constexpr int MI = MG_TILE / MG_THREADS;
    static_assert(MI <= 4 && MG_THREADS < 65536, "flags are packed 16 bits per round");
    (void)ta;
    const int64_t nb = (R + MG_TILE - 1) / MG_TILE;
    const uint32_t tb32 = (uint32_t)tb;
    const double inv_tb = 1.0 / (double)tb;
    // mixed-radix key -> bit fields of dec.bits bits (the unpack kernel's
    // layout), least significant digit first: chunks of dec.chunk digits
    // (radix^chunk < 2^32) split off by one 64-bit division, then the digits
    // of a chunk by 32-bit divisions.  Each quotient comes from the high half
    // of a product with floor((2^w - 1) / divisor), which is exact or one
    // short, and is corrected.
    auto to_fields = [&](uint64_t x) {
        uint64_t f = 0;
        const uint32_t r = (uint32_t)dec.radix;
        for (int i = 0; i < dec.n; i += dec.chunk) {
            uint32_t lo;
            if (dec.n - i > dec.chunk) {
                uint64_t q = __umul64hi(x, dec.div_magic);
                uint64_t rem = x - q * dec.div;
                if (rem >= dec.div) {
                    ++q;
                    rem -= dec.div;
                }
                lo = (uint32_t)rem;
                x = q;
            } else {
                lo = (uint32_t)x;
            }
            const int e = dec.n - i < dec.chunk ? dec.n - i : dec.chunk;
            for (int j = 0; j < e; ++j) {
                uint32_t q = __umulhi(lo, dec.digit_magic);
                uint32_t rem = lo - q * r;
                if (rem >= r) {
                    ++q;
                    rem -= r;
                }
                f |= (uint64_t)rem << (dec.bits * (i + j));
                lo = q;
            }
        }
        return f;
    };
    auto split_raw = [&](uint32_t r) {
        // r / tb in double precision (within one of the quotient for 32-bit r), then corrected
        uint32_t i = (uint32_t)((double)r * inv_tb);
        if (i * (uint64_t)tb32 > r) --i;
        else if ((uint64_t)(i + 1) * tb32 <= r) ++i;
        return make_uint2(i, r - i * tb32);
    };
    auto product = [&](uint32_t r) {
        const uint2 ij = split_raw(r);
        return ca[ij.x] * cb[ij.y];
    };
    const uint64_t rmask = raw_bits >= 64 ? ~0ull : ((1ull << raw_bits) - 1ull);
    // key and raw index of element g of the sorted stream
    auto element = [&](int64_t g, uint32_t &raw) -> uint64_t {
        if (PACKED) {
            raw = (uint32_t)(keys[g] & rmask);
            const uint2 ij = split_raw(raw);
            return ka[ij.x] + kb[ij.y];
        }
        raw = vals[g];
        return keys[g];
    };
    // the elements of the next tile are loaded while the current one is
    // merged (issued after its coefficient gathers, so waiting on those never
    // waits on them)
    uint64_t kn[MI];
    uint32_t vn[MI];
    auto load_tile = [&](int64_t blk) {
        const int64_t t0 = blk * MG_TILE;
        const int m = (int)(R - t0 < MG_TILE ? R - t0 : MG_TILE);
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * MG_THREADS + threadIdx.x;
            const int lc = l < m ? l : m - 1;
            kn[q] = keys[t0 + lc];
            vn[q] = PACKED ? 0u : vals[t0 + lc];
        }
    };
    if ((int64_t)blockIdx.x < nb) load_tile(blockIdx.x);
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int64_t t0 = blk * MG_TILE;
        const int m = (int)(R - t0 < MG_TILE ? R - t0 : MG_TILE);
        // halo: up to GS_HALO elements after the tile, where its last run
        // usually ends
        const int hl = (int)(R - t0 - m < GS_HALO ? R - t0 - m : GS_HALO);
        __syncthreads();   // the previous tile's LDS reads are done
        uint64_t kr[MI + 1];
        uint32_t vr[MI + 1];
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            kr[q] = kn[q];
            vr[q] = vn[q];
        }
        {
            const int hc = threadIdx.x < hl ? (int)threadIdx.x : 0;
            kr[MI] = hl > 0 ? keys[t0 + m + hc] : 0ull;
            vr[MI] = (!PACKED && hl > 0) ? vals[t0 + m + hc] : 0u;
        }
        uint32_t rb_;
        const uint64_t before = (threadIdx.x == 0 && t0 > 0) ? element(t0 - 1, rb_) : 0ull;
        double ci[MI + 1], cj[MI + 1];
#pragma unroll
        for (int q = 0; q <= MI; ++q) {
            ci[q] = cj[q] = 0.0;
            if (q == MI && threadIdx.x >= kWave) break;   // the halo is the first wave's
            if (PACKED) vr[q] = (uint32_t)(kr[q] & rmask);
            const uint2 ij = split_raw(vr[q]);
            if (PACKED) {   // key and coefficient of each factor in one gather
                const GsKC x = pa[ij.x], y = pb[ij.y];
                ci[q] = x.c;
                cj[q] = y.c;
                kr[q] = x.k + y.k;
            } else {
                ci[q] = ca[ij.x];
                cj[q] = cb[ij.y];
            }
        }
        if (blk + (int64_t)gridDim.x < nb) load_tile(blk + gridDim.x);
#pragma unroll
        for (int q = 0; q < MI; ++q) {
            const int l = q * MG_THREADS + threadIdx.x;
            if (l < m) {
                s_key[l] = kr[q];
                s_prod[l] = ci[q] * cj[q];
            }
        }
        if ((int)threadIdx.x < hl) {
            s_key[m + threadIdx.x] = kr[MI];
            s_prod[m + threadIdx.x] = ci[MI] * cj[MI];
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
                double s = s_prod[l];
                for (int f = l + 1; f < e; ++f) s = s + s_prod[f];
                if (k == nh - 1) {
                    // the run may continue past the tile: the halo, then
                    // (runs longer than it) the stream itself
                    int f = m;
                    for (; f < m + hl && s_key[f] == key; ++f) s = s + s_prod[f];
                    if (f == m + hl)
                        for (int64_t g = t0 + m + hl; g < R; ++g) {
                            uint32_t rg;
                            if (element(g, rg) != key) break;
                            s = s + product(rg);
                        }
                }
                if (!(fabs(s) <= tol)) {
                    hk[q] = to_fields(key);
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

#define GS_SCATTER_INST(DB, MODE)                                                                              \
    template __global__ void k_gs_scatter<DB, MODE>(const uint64_t *, const uint32_t *, int64_t, int, int64_t,     \
                                                    const int64_t *, uint64_t *, uint32_t *, int,                   \
                                                    unsigned long long *, int64_t, GsGen);
#define GS_DIGIT_INST(DB)                                                                                      \
    template __global__ void k_gs_hist<DB, false>(const uint64_t *, int64_t, int, int64_t, int64_t *, GsGen);   \
    template __global__ void k_gs_hist<DB, true>(const uint64_t *, int64_t, int, int64_t, int64_t *, GsGen);    \
    GS_SCATTER_INST(DB, GS_KV)                                                                                  \
    GS_SCATTER_INST(DB, GS_KV_TO_PACKED)                                                                        \
    GS_SCATTER_INST(DB, GS_PACKED)                                                                              \
    GS_SCATTER_INST(DB, GS_GEN_KV)                                                                              \
    GS_SCATTER_INST(DB, GS_GEN_TO_PACKED)
GS_DIGIT_INST(4)
GS_DIGIT_INST(5)
GS_DIGIT_INST(6)
GS_DIGIT_INST(7)
GS_DIGIT_INST(8)
GS_DIGIT_INST(9)
GS_DIGIT_INST(10)
GS_DIGIT_INST(11)
#undef GS_DIGIT_INST
#undef GS_SCATTER_INST
template __global__ void k_gs_merge<false>(const uint64_t *, const uint32_t *, int64_t, int64_t, int64_t,
                                           const uint64_t *, const uint64_t *, int, const double *,
                                           const double *, const GsKC *, const GsKC *, double, RadixDecode,
                                           uint64_t *, double *, int64_t *, int64_t *);
template __global__ void k_gs_merge<true>(const uint64_t *, const uint32_t *, int64_t, int64_t, int64_t,
                                          const uint64_t *, const uint64_t *, int, const double *,
                                          const double *, const GsKC *, const GsKC *, double, RadixDecode,
                                          uint64_t *, double *, int64_t *, int64_t *);

__global__ void k_gs_pairs(const uint64_t *keys, const double *coefs, int64_t T, GsKC *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) out[t] = GsKC{keys[t], coefs[t]};
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
