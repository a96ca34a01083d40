// Internal device/host helpers shared by the polyhip HIP sources.
// gfx950 only: wave64, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/polyhip.h"

namespace polyhip {

constexpr int kWave = 64;

// First 256 bytes of every workspace: the device status word.
struct WsHead {
    int32_t status;
    int32_t pad[63];
};
constexpr size_t kWsHeadBytes = 256;

__device__ inline void set_status(int32_t *st, int32_t code)
{
    atomicMax(st, code);
}

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Inclusive prefix sum across the 64 lanes of a wave.
template <class T>
__device__ inline T wave_inclusive_scan(T x)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

template <class T>
__device__ inline T wave_sum(T x)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// Block-wide exclusive scan; `scratch` holds THREADS/64 elements.  Every
// thread of the block must call it.  Returns the exclusive prefix; `total`
// receives the block sum.
template <int THREADS, class T>
__device__ inline T block_exclusive_scan(T v, T *scratch, T &total)
{
    constexpr int W = THREADS / kWave;
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) scratch[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        T s = scratch[i];
        off += (i < w) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

template <int THREADS, class T>
__device__ inline T block_sum(T v, T *scratch)
{
    T tot;
    (void)block_exclusive_scan<THREADS>(v, scratch, tot);
    return tot;
}

template <int THREADS>
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t *scratch)
{
    constexpr int W = THREADS / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(v, o, kWave);
        v = y < v ? y : v;
    }
    if (lane_id() == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t r = scratch[0];
#pragma unroll
    for (int i = 1; i < W; ++i) r = scratch[i] < r ? scratch[i] : r;
    __syncthreads();
    return r;
}

template <int THREADS>
__device__ inline uint64_t block_max_u64(uint64_t v, uint64_t *scratch)
{
    constexpr int W = THREADS / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(v, o, kWave);
        v = y > v ? y : v;
    }
    if (lane_id() == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t r = scratch[0];
#pragma unroll
    for (int i = 1; i < W; ++i) r = scratch[i] > r ? scratch[i] : r;
    __syncthreads();
    return r;
}

// Bit width needed to hold v (v = 0 -> 1).
__host__ __device__ inline int bit_width_u32(uint32_t v)
{
    int b = 1;
    while ((v >> b) != 0) ++b;
    return b;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// 32-bit integer hash (xorshift-multiply) for deterministic sampling.
__device__ inline uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

}  // namespace polyhip
