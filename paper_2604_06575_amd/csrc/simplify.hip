// simplify (Table "coresemantics": merge repeated monomials, drop small
// coefficients) as a persistent segmented sort-and-merge over a CSR batch.
//
// Every exponent row is packed into a 64-bit key (b bits per variable, x1 in
// the most significant field), so ascending key order is the canonical
// lexicographic order.  One workgroup takes one entry at a time from an
// atomic job counter (entries ordered largest first).  An entry that fits in
// LDS is sorted there as (key, local index) pairs, which orders equal keys by
// their position in the input; each run of equal keys is then summed left to
// right by one lane, exactly the order of a sequential merge.  Larger entries
// are cut into key ranges by bisection until each range fits in LDS.
#pragma clang fp contract(off)

#include "kernels.h"
#include "lds_sort.h"

namespace polyhip {

__global__ void k_pack(const uint8_t *__restrict__ exps, int64_t T, int n, int bits, int max_exp,
                       uint64_t *__restrict__ keys, int32_t *status)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint8_t *row = exps + t * n;
    uint64_t k = 0;
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t e = row[i];
        bad |= (int)(e > (uint32_t)max_exp);
        k = (k << bits) | (uint64_t)e;
    }
    keys[t] = k;
    if (bad) set_status(status, POLY_ERR_EXPONENT);
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Entries ordered by decreasing size class (floor(log2(size))); one block.
__global__ void __launch_bounds__(1024) k_order_by_size(const int64_t *rp, int64_t P, int64_t *order)
{
    __shared__ int64_t s_hist[66];
    __shared__ int64_t s_cur[66];
    for (int i = threadIdx.x; i < 66; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        const int64_t sz = rp[p + 1] - rp[p];
        const int cls = sz <= 0 ? 0 : 64 - __clzll((unsigned long long)sz);  // 1..64
        atomicAdd((unsigned long long *)&s_hist[65 - cls], 1ull);              // largest class first
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int c = 0; c < 66; ++c) {
            s_cur[c] = run;
            run += s_hist[c];
        }
    }
    __syncthreads();
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        const int64_t sz = rp[p + 1] - rp[p];
        const int cls = sz <= 0 ? 0 : 64 - __clzll((unsigned long long)sz);
        const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&s_cur[65 - cls], 1ull);
        order[pos] = p;
    }
}

namespace {

struct SegShared {
    uint64_t key[SEG_CAP];
    uint32_t val[SEG_CAP];
    uint32_t cnt[(SEG_THREADS / kWave) * 256];
    uint32_t scan32[SEG_THREADS / kWave];
    int64_t scan[SEG_THREADS / kWave];
    uint64_t red[SEG_THREADS / kWave];
    uint64_t stk_lo[72];
    uint64_t stk_hi[72];
    int64_t stk_cnt[72];
    int64_t job;
    double bcast;
    int64_t bcast_i;
};

// Sort the tile's m (key, local index) pairs by key.  The elements are in
// storage order, and the radix sort is stable, so equal keys stay in storage
// order.  Keys are made relative to the tile minimum so that only the bits
// that actually vary are sorted.
__device__ void sort_tile(SegShared &S, int m)
{
    uint64_t lmin = ~0ull, lmax = 0;
    for (int i = threadIdx.x; i < m; i += SEG_THREADS) {
        const uint64_t k = S.key[i];
        lmin = k < lmin ? k : lmin;
        lmax = k > lmax ? k : lmax;
    }
    const uint64_t kmin = block_min_u64<SEG_THREADS>(lmin, S.red);
    const uint64_t kmax = block_max_u64<SEG_THREADS>(lmax, S.red);
    if (m == 0) return;
    for (int i = threadIdx.x; i < m; i += SEG_THREADS) S.key[i] -= kmin;
    __syncthreads();
    const int bits = kmax > kmin ? 64 - __clzll((unsigned long long)(kmax - kmin)) : 0;
    lds_radix_sort<SEG_THREADS, SEG_ITEMS>(S.key, S.val, m, bits, S.cnt, S.scan32);
    for (int i = threadIdx.x; i < m; i += SEG_THREADS) S.key[i] += kmin;
    __syncthreads();
}

// Emit the sorted tile: merged runs (merge mode) or every element (sort mode)
// to staging positions base + out .. ; returns the number written.
template <bool SORT_ONLY>
__device__ int64_t emit_tile(const SegArgs &A, SegShared &S, int m, int64_t base, int64_t out)
{
    if (SORT_ONLY) {
        for (int i = threadIdx.x; i < m; i += SEG_THREADS) {
            A.st_key[base + out + i] = S.key[i];
            A.st_idx[base + out + i] = S.val[i];
        }
        __syncthreads();
        return m;
    }
    int64_t written = 0;
    for (int c0 = 0; c0 < m; c0 += SEG_THREADS) {
        const int i = c0 + threadIdx.x;
        int64_t keep = 0;
        double s = 0.0;
        uint64_t k = 0;
        if (i < m) {
            k = S.key[i];
            const bool head = (i == 0) || (S.key[i - 1] != k);
            if (head) {
                s = A.coefs[base + S.val[i]];
                for (int q = i + 1; q < m && S.key[q] == k; ++q) s = s + A.coefs[base + S.val[q]];
                keep = !(fabs(s) <= A.tol);
            }
        }
        int64_t tot;
        const int64_t pos = block_exclusive_scan<SEG_THREADS>(keep, S.scan, tot);
        if (keep) {
            A.st_key[base + out + written + pos] = k;
            A.st_coef[base + out + written + pos] = s;
        }
        written += tot;
    }
    return written;
}

template <bool SORT_ONLY>
__device__ void seg_process(const SegArgs &A, SegShared &S)
{
    for (;;) {
        if (threadIdx.x == 0) S.job = (int64_t)atomicAdd(A.queue, 1ull);
        __syncthreads();
        const int64_t job = S.job;
        __syncthreads();
        if (job >= A.P) break;
        const int64_t p = A.order[job];
        const int64_t base = A.rp[p];
        const int64_t T = A.rp[p + 1] - base;
        int64_t written = 0;
        if (T <= SEG_CAP) {
            for (int i = threadIdx.x; i < T; i += SEG_THREADS) {
                S.key[i] = A.keys[base + i];
                S.val[i] = (uint32_t)i;
            }
            __syncthreads();
            sort_tile(S, (int)T);
            written = emit_tile<SORT_ONLY>(A, S, (int)T, base, 0);
        } else {
            uint64_t lmin = ~0ull, lmax = 0;
            for (int64_t i = threadIdx.x; i < T; i += SEG_THREADS) {
                const uint64_t k = A.keys[base + i];
                lmin = k < lmin ? k : lmin;
                lmax = k > lmax ? k : lmax;
            }
            const uint64_t kmin = block_min_u64<SEG_THREADS>(lmin, S.red);
            const uint64_t kmax = block_max_u64<SEG_THREADS>(lmax, S.red);
            if (threadIdx.x == 0) {
                S.stk_lo[0] = kmin;
                S.stk_hi[0] = kmax;
                S.stk_cnt[0] = T;
            }
            int sp = 1;
            while (sp > 0) {
                __syncthreads();
                --sp;
                const uint64_t lo = S.stk_lo[sp], hi = S.stk_hi[sp];
                const int64_t cnt = S.stk_cnt[sp];
                __syncthreads();
                if (cnt == 0) continue;
                if (cnt <= SEG_CAP) {
                    // stable gather of the range into LDS
                    int64_t got = 0;
                    for (int64_t c0 = 0; c0 < T; c0 += SEG_THREADS) {
                        const int64_t i = c0 + threadIdx.x;
                        int64_t f = 0;
                        uint64_t k = 0;
                        if (i < T) {
                            k = A.keys[base + i];
                            f = (k >= lo && k <= hi) ? 1 : 0;
                        }
                        int64_t tot;
                        const int64_t pos = block_exclusive_scan<SEG_THREADS>(f, S.scan, tot);
                        if (f && got + pos < SEG_CAP) {
                            S.key[got + pos] = k;
                            S.val[got + pos] = (uint32_t)i;
                        }
                        got += tot;
                    }
                    const int m = (int)(got < SEG_CAP ? got : SEG_CAP);
                    __syncthreads();
                    sort_tile(S, m);
                    written += emit_tile<SORT_ONLY>(A, S, m, base, written);
                } else if (lo == hi) {
                    // one key repeated more often than a tile holds
                    if (SORT_ONLY) {
                        int64_t got = 0;
                        for (int64_t c0 = 0; c0 < T; c0 += SEG_THREADS) {
                            const int64_t i = c0 + threadIdx.x;
                            int64_t f = (i < T && A.keys[base + i] == lo) ? 1 : 0;
                            int64_t tot;
                            const int64_t pos = block_exclusive_scan<SEG_THREADS>(f, S.scan, tot);
                            if (f) {
                                A.st_key[base + written + got + pos] = lo;
                                A.st_idx[base + written + got + pos] = (uint32_t)i;
                            }
                            got += tot;
                        }
                        written += got;
                    } else {
                        if (threadIdx.x == 0) {
                            double s = 0.0;
                            bool first = true;
                            for (int64_t i = 0; i < T; ++i) {
                                if (A.keys[base + i] != lo) continue;
                                const double c = A.coefs[base + i];
                                s = first ? c : s + c;
                                first = false;
                            }
                            const bool keep = !(fabs(s) <= A.tol);
                            if (keep) {
                                A.st_key[base + written] = lo;
                                A.st_coef[base + written] = s;
                            }
                            S.bcast_i = keep ? 1 : 0;
                        }
                        __syncthreads();
                        written += S.bcast_i;
                        __syncthreads();
                    }
                } else {
                    const uint64_t mid = lo + (hi - lo) / 2;
                    int64_t c = 0;
                    for (int64_t i = threadIdx.x; i < T; i += SEG_THREADS) {
                        const uint64_t k = A.keys[base + i];
                        c += (k >= lo && k <= mid) ? 1 : 0;
                    }
                    const int64_t left = block_sum<SEG_THREADS>(c, S.scan);
                    if (threadIdx.x == 0) {
                        S.stk_lo[sp] = mid + 1;
                        S.stk_hi[sp] = hi;
                        S.stk_cnt[sp] = cnt - left;
                        S.stk_lo[sp + 1] = lo;
                        S.stk_hi[sp + 1] = mid;
                        S.stk_cnt[sp + 1] = left;
                    }
                    sp += 2;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) A.seg_count[p] = written;
        __syncthreads();
    }
}

}  // namespace

__global__ void __launch_bounds__(SEG_THREADS) k_seg_merge(SegArgs A)
{
    __shared__ SegShared S;
    seg_process<false>(A, S);
}

__global__ void __launch_bounds__(SEG_THREADS) k_seg_sort(SegArgs A)
{
    __shared__ SegShared S;
    seg_process<true>(A, S);
}

// Two independent segment sets in one launch (both operands of a product);
// the blocks split the machine between them.
__global__ void __launch_bounds__(SEG_THREADS) k_seg_sort2(SegArgs A, SegArgs B)
{
    __shared__ SegShared S;
    if (blockIdx.x & 1) seg_process<true>(B, S);
    else seg_process<true>(A, S);
}

// Exclusive scan of S counts into out[0..S]; one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan_counts(const int64_t *counts, int64_t S, int64_t *out)
{
    __shared__ int64_t s_scan[1024 / kWave];
    int64_t run = 0;
    for (int64_t c0 = 0; c0 < S; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < S ? counts[i] : 0;
        int64_t tot;
        const int64_t pos = block_exclusive_scan<1024>(v, s_scan, tot);
        if (i < S) out[i] = run + pos;
        run += tot;
    }
    if (threadIdx.x == 0) out[S] = run;
}

// Single-pass exclusive scan with decoupled look-back (Merrill and Garland).
// Tiles are taken in the order workgroups start (a ticket), so every tile's
// predecessors are running or done and the look-back always ends.  A tile
// publishes its sum as soon as it is known (status AGG), then its inclusive
// prefix (status PFX) once its look-back is done; the look-back reads 64
// predecessors per round, one per lane, and adds them up to the nearest PFX.
// Status and value share one 64-bit word.  out[S] = total.  The state must be
// zero on entry; the scan leaves it dirty (the caller clears it, in a later
// kernel, before the next scan).
namespace {
constexpr unsigned long long LB_AGG = 1ull << 62, LB_PFX = 2ull << 62, LB_VAL = (1ull << 62) - 1;
}

__global__ void __launch_bounds__(LB_THREADS) k_scan_lookback(const int64_t *in, int64_t S, int64_t *out,
                                                                unsigned long long *state, int32_t *status)
{
    __shared__ int64_t s_scan[LB_THREADS / kWave];
    __shared__ int64_t s_excl;
    __shared__ int64_t s_tile;
    unsigned long long *flag = state + 2;
    const int64_t nt = (S + LB_TILE - 1) / LB_TILE;
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(&state[0], 1ull);
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= nt) {   // state not zero on entry: a caller bug, reported rather than waited on
        if (threadIdx.x == 0) set_status(status, POLY_ERR_HIP);
        return;
    }
    const int64_t i0 = t * LB_TILE + (int64_t)threadIdx.x * LB_ITEMS;
    int64_t v[LB_ITEMS];
    int64_t loc = 0;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        const int64_t i = i0 + k;
        v[k] = in[i < S ? i : S - 1];
    }
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        v[k] = i0 + k < S ? v[k] : 0;
        loc += v[k];
    }
    int64_t tot;
    const int64_t pos = block_exclusive_scan<LB_THREADS>(loc, s_scan, tot);
    if (threadIdx.x == 0)
        __hip_atomic_store(&flag[t], (t == 0 ? LB_PFX : LB_AGG) | (unsigned long long)tot, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < kWave) {
        const int lane = (int)threadIdx.x;
        int64_t excl = 0;
        int64_t j = t - 1;   // nearest predecessor not yet added
        uint32_t spins = 0;  // bounded: predecessors never wait on this tile, so a limit means a bug
        while (j >= 0) {
            const int64_t jj = j - lane;
            const unsigned long long f =
                jj >= 0 ? __hip_atomic_load(&flag[jj], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_PFX;
            const unsigned long long pfx = __ballot((f >> 62) == 2ull);
            const unsigned long long none = __ballot((f >> 62) == 0ull);
            // lanes up to the nearest PFX lane must all have published
            const int stop = pfx ? __ffsll((long long)pfx) - 1 : kWave - 1;
            const unsigned long long upto = stop == kWave - 1 ? ~0ull : ((1ull << (stop + 1)) - 1);
            if (none & upto) {   // a predecessor still working: read again
                if (++spins > (1u << 22)) {
                    if (lane == 0) set_status(status, POLY_ERR_HIP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            int64_t part = lane <= stop ? (int64_t)(f & LB_VAL) : 0;
            part = wave_sum(part);
            excl += part;
            if (pfx) break;
            j -= kWave;
        }
        if (lane == 0) {
            s_excl = excl;
            if (t > 0)
                __hip_atomic_store(&flag[t], LB_PFX | (unsigned long long)(excl + tot), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    int64_t run = s_excl + pos;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        const int64_t i = i0 + k;
        if (i < S) out[i] = run;
        run += v[k];
    }
    if (t == nt - 1 && threadIdx.x == 0) out[S] = s_excl + tot;
}

// One block per segment: staged (key, coef) -> CSR output rows.  A segment's
// output rows are contiguous, so its exponent bytes form one contiguous
// range; the block writes that range as aligned 32-bit words (each byte
// unpacked from its row's key), with the unaligned head and tail bytes
// written singly, so neighbouring segments never share a store.
__global__ void __launch_bounds__(256) k_compact(const int64_t *stage_off, const int64_t *seg_count,
                                                 const int64_t *out_off, const uint64_t *st_key,
                                                 const double *st_coef, int n, int bits, uint8_t *out_exps,
                                                 double *out_coefs, int64_t capacity, int32_t *status)
{
    const int64_t s = blockIdx.x;
    const int64_t cnt = seg_count[s];
    const int64_t src = stage_off[s];
    const int64_t dst = out_off[s];
    if (threadIdx.x == 0 && dst + cnt > capacity) set_status(status, POLY_ERR_CAPACITY);
    const int64_t end = dst + cnt < capacity ? dst + cnt : capacity;
    if (end <= dst) return;
    for (int64_t i = dst + threadIdx.x; i < end; i += blockDim.x) out_coefs[i] = st_coef[src + (i - dst)];
    const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1ull);
    const int64_t b0 = dst * n, b1 = end * n;
    int64_t w0 = (b0 + 3) & ~(int64_t)3, w1 = b1 & ~(int64_t)3;
    if (w0 > b1) w0 = b1;
    if (w1 < w0) w1 = w0;
    const uint32_t un = (uint32_t)n;
    const uint64_t *keys = st_key + src;
    // byte bi (absolute) -> row (bi - b0) / n of this segment, field (bi - b0) % n
    auto byte_at = [&](int64_t bi) -> uint32_t {
        const uint32_t rel = (uint32_t)(bi - b0);
        const uint32_t row = rel / un, f = rel - row * un;
        return (uint32_t)((keys[row] >> (bits * (n - 1 - (int)f))) & mask);
    };
    for (int64_t bi = b0 + threadIdx.x; bi < w0; bi += blockDim.x) out_exps[bi] = (uint8_t)byte_at(bi);
    for (int64_t bi = w1 + threadIdx.x; bi < b1; bi += blockDim.x) out_exps[bi] = (uint8_t)byte_at(bi);
    uint32_t *words = (uint32_t *)out_exps;
    for (int64_t w = w0 / 4 + threadIdx.x; w < w1 / 4; w += blockDim.x) {
        const uint32_t rel = (uint32_t)(w * 4 - b0);
        uint32_t row = rel / un;
        uint32_t f = rel - row * un;
        uint64_t k = keys[row];
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (f == un) {
                f = 0;
                ++row;
                k = keys[row];
            }
            v |= (uint32_t)((k >> (bits * (n - 1 - (int)f))) & mask) << (8 * q);
            ++f;
        }
        words[w] = v;
    }
}

}  // namespace polyhip
