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
