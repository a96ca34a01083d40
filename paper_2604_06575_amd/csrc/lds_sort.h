// Block-wide sorts of (u64 key, u32 payload) pairs held in LDS.
//
// Order is (key, payload) lexicographic, ascending.  Payloads are unique
// within a tile (a term index or a product pair index), so the result is the
// stable order of the keys with respect to the payload: this is what makes the
// later run sums follow the raw term order exactly.
#pragma once

#include "internal.h"

namespace polyhip {

__device__ inline bool kv_greater(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb)
{
    return (ka > kb) || (ka == kb && va > vb);
}

// Sort keys[0..m) / vals[0..m) in place; M = next power of two >= m must fit
// in the arrays (slots [m, M) are overwritten with +inf padding).
template <int THREADS>
__device__ void lds_sort_kv(uint64_t *keys, uint32_t *vals, int m)
{
    int M = 1;
    while (M < m) M <<= 1;
    for (int i = m + threadIdx.x; i < M; i += THREADS) {
        keys[i] = ~0ull;
        vals[i] = ~0u;
    }
    __syncthreads();
    if (M < 2) return;
    // Stages with j >= 64 go through LDS with a barrier; the tail of each
    // merge level (j < 64 pairs within a 128-element window) is still done
    // in LDS but needs no barrier between sub-stages when one wave owns the
    // whole window; kept simple here: a barrier after every stage.
    for (int k = 2; k <= M; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < (M >> 1); i += THREADS) {
                const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int b = a + j;
                const uint64_t ka = keys[a], kb = keys[b];
                const uint32_t va = vals[a], vb = vals[b];
                const bool up = (a & k) == 0;
                if (kv_greater(ka, va, kb, vb) == up) {
                    keys[a] = kb;
                    keys[b] = ka;
                    vals[a] = vb;
                    vals[b] = va;
                }
            }
            __syncthreads();
        }
    }
}

// Keys only (used for sample sorts).
template <int THREADS>
__device__ void lds_sort_keys(uint64_t *keys, int m)
{
    int M = 1;
    while (M < m) M <<= 1;
    for (int i = m + threadIdx.x; i < M; i += THREADS) keys[i] = ~0ull;
    __syncthreads();
    if (M < 2) return;
    for (int k = 2; k <= M; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < (M >> 1); i += THREADS) {
                const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int b = a + j;
                const uint64_t ka = keys[a], kb = keys[b];
                const bool up = (a & k) == 0;
                if ((ka > kb) == up) {
                    keys[a] = kb;
                    keys[b] = ka;
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace polyhip

namespace polyhip {

// Stable LSD radix sort (8-bit digits) of (u64 key, u32 payload) pairs held in
// LDS, ascending by the low `key_bits` bits of the key (higher bits must be
// equal across the tile, e.g. keys made relative to the tile minimum).
// Elements [0, m) are valid, m <= THREADS * ITEMS; the arrays must hold
// THREADS * ITEMS slots (the tail is used as +inf padding).  Wave w owns the
// contiguous element chunk [w*64*ITEMS, (w+1)*64*ITEMS) and reads it in rounds
// of 64 lanes, so (wave, round, lane) is the input order; equal digits keep
// that order (lane ranks from wavefront ballots, earlier rounds and waves from
// LDS counters), which makes every pass stable.
// s_cnt holds (THREADS/64) * 256 counters; s_scan THREADS/64 words.
template <int THREADS, int ITEMS, class V = uint32_t>
__device__ void lds_radix_sort(uint64_t *keys, V *vals, int m, int key_bits, uint32_t *s_cnt, uint32_t *s_scan)
{
    constexpr int W = THREADS / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x >> 6;
    const unsigned long long lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    for (int sh = 0; sh < key_bits; sh += 8) {
        uint64_t k[ITEMS];
        V v[ITEMS];
        uint32_t pos[ITEMS];
        uint32_t dg[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int e = (w * ITEMS + it) * kWave + lane;
            if (e < m) {
                k[it] = keys[e];
                v[it] = vals[e];
            } else {
                k[it] = ~0ull;
                v[it] = V(0);
            }
            dg[it] = (uint32_t)((k[it] >> sh) & 0xffu);
        }
        for (int i = threadIdx.x; i < W * 256; i += THREADS) s_cnt[i] = 0;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t d = dg[it];
            unsigned long long peer = ~0ull;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const unsigned long long bb = __ballot(bit);
                peer &= bit ? bb : ~bb;
            }
            const uint32_t prior = s_cnt[w * 256 + d];
            pos[it] = prior + (uint32_t)__popcll(peer & lt);
            if ((peer & lt) == 0) s_cnt[w * 256 + d] = prior + (uint32_t)__popcll(peer);
        }
        __syncthreads();
        // exclusive scan over (digit, wave), digit-major
        uint32_t pre[W];
        uint32_t tot = 0;
        if (threadIdx.x < 256) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                pre[ww] = tot;
                tot += s_cnt[ww * 256 + threadIdx.x];
            }
        }
        uint32_t all;
        const uint32_t base = block_exclusive_scan<THREADS>(threadIdx.x < 256 ? tot : 0u, s_scan, all);
        if (threadIdx.x < 256) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) s_cnt[ww * 256 + threadIdx.x] = base + pre[ww];
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t p = s_cnt[w * 256 + dg[it]] + pos[it];
            keys[p] = k[it];
            vals[p] = v[it];
        }
        __syncthreads();
    }
}

}  // namespace polyhip

namespace polyhip {

// Keys-only variant of lds_radix_sort (same ordering rules).
template <int THREADS, int ITEMS>
__device__ void lds_radix_sort_keys(uint64_t *keys, int m, int key_bits, uint32_t *s_cnt, uint32_t *s_scan)
{
    constexpr int W = THREADS / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x >> 6;
    const unsigned long long lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    for (int sh = 0; sh < key_bits; sh += 8) {
        uint64_t k[ITEMS];
        uint32_t pos[ITEMS];
        uint32_t dg[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int e = (w * ITEMS + it) * kWave + lane;
            k[it] = e < m ? keys[e] : ~0ull;
            dg[it] = (uint32_t)((k[it] >> sh) & 0xffu);
        }
        for (int i = threadIdx.x; i < W * 256; i += THREADS) s_cnt[i] = 0;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t d = dg[it];
            unsigned long long peer = ~0ull;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const unsigned long long bb = __ballot(bit);
                peer &= bit ? bb : ~bb;
            }
            const uint32_t prior = s_cnt[w * 256 + d];
            pos[it] = prior + (uint32_t)__popcll(peer & lt);
            if ((peer & lt) == 0) s_cnt[w * 256 + d] = prior + (uint32_t)__popcll(peer);
        }
        __syncthreads();
        uint32_t pre[W];
        uint32_t tot = 0;
        if (threadIdx.x < 256) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                pre[ww] = tot;
                tot += s_cnt[ww * 256 + threadIdx.x];
            }
        }
        uint32_t all;
        const uint32_t base = block_exclusive_scan<THREADS>(threadIdx.x < 256 ? tot : 0u, s_scan, all);
        if (threadIdx.x < 256) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) s_cnt[ww * 256 + threadIdx.x] = base + pre[ww];
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) keys[s_cnt[w * 256 + dg[it]] + pos[it]] = k[it];
        __syncthreads();
    }
}

}  // namespace polyhip
