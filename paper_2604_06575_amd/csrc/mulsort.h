// Global radix-sort path of times + simplify for one large pair
// (mulsort.hip): launch constants and kernels.
#pragma once
#include "internal.h"

namespace polyhip {

constexpr int GS_THREADS = 1024;                 // operand sort, raw product generation
constexpr int GS_SC_THREADS = 512;               // radix-pass (scatter) workgroup
constexpr int GS_ITEMS = 8;
constexpr int GS_TILE = GS_SC_THREADS * GS_ITEMS;   // elements per scatter workgroup and pass
constexpr int GS_MAX_BITS = 11;                  // widest digit instantiated
constexpr int GS_MIN_BITS = 4;                   // narrowest digit instantiated
constexpr int GS_HIST_THREADS = 256;
constexpr int MG_THREADS = 512;                  // merge workgroup
constexpr int MG_TILE = MG_THREADS * 4;          // merge elements per tile
constexpr int MG_BLOCKS_PER_CU = 4;              // persistent merge workgroups per CU
constexpr int GS_HALO = 64;                      // elements past a tile staged by the merge
__global__ void k_gs_pack_radix(const uint8_t *exps, int64_t T, int n, uint64_t radix, int max_exp,
                                uint64_t *keys, int32_t *status);
__global__ void k_gs_generate(const uint64_t *ka, const uint64_t *kb, int64_t ta, int64_t tb, uint64_t *keys,
                              uint32_t *vals);
// Elements of the raw product in raw order, generated instead of read: the
// element with raw index r = i * tb + j has key ka[i] + kb[j].  The first
// radix pass and its histogram read the product this way, so it is never
// written to memory.
struct GsGen {
    const uint64_t *ka;
    const uint64_t *kb;
    uint32_t tb;
    double inv_tb;   // 1 / tb
    // A lane's elements in a radix pass are raw indices in increasing order,
    // at most one wavefront (64) apart: the first one's (i, j) is found by
    // division, and from it on (i, j) steps forward without one whenever
    // tb >= 64 (one row end at most per step).
    struct Cursor {
        uint32_t i, j, r;
    };
    __device__ uint64_t first(uint32_t r, Cursor &c) const
    {
        // r / tb in double precision (within one of the quotient for 32-bit r), then corrected
        uint32_t i = (uint32_t)((double)r * inv_tb);
        if (i * (uint64_t)tb > r) --i;
        else if ((uint64_t)(i + 1) * tb <= r) ++i;
        c.i = i;
        c.j = r - i * tb;
        c.r = r;
        return ka[c.i] + kb[c.j];
    }
    __device__ uint64_t next(uint32_t r, Cursor &c) const   // r >= c.r, r - c.r <= 64
    {
        if (tb < 64) return first(r, c);
        c.j += r - c.r;
        c.r = r;
        if (c.j >= tb) {
            c.j -= tb;
            ++c.i;
        }
        return ka[c.i] + kb[c.j];
    }
};

template <int DB, bool GEN>
__global__ void k_gs_hist(const uint64_t *keys, int64_t R, int shift, int64_t nblocks, int64_t *hist, GsGen gen);
// element formats of a radix pass
enum { GS_KV = 0, GS_KV_TO_PACKED = 1, GS_PACKED = 2, GS_GEN_KV = 3, GS_GEN_TO_PACKED = 4 };
template <int DB, int MODE>
__global__ void k_gs_scatter(const uint64_t *keys_in, const uint32_t *vals_in, int64_t R, int shift,
                             int64_t nblocks, const int64_t *hist_off, uint64_t *keys_out, uint32_t *vals_out,
                             int raw_bits, unsigned long long *clear, int64_t clear_n, GsGen gen);
// Division constants for turning mixed-radix keys back into bit fields.
struct RadixDecode {
    uint64_t radix;         // r
    uint64_t div;           // r^chunk (< 2^32)
    uint64_t div_magic;     // floor((2^64 - 1) / div)
    uint32_t digit_magic;   // floor((2^32 - 1) / r)
    int chunk;              // digits per 64-bit division, 1 <= chunk <= n
    int n;                  // digits (variables)
    int bits;               // output field width
};
// an operand term's key and coefficient side by side (one 16-byte gather)
struct __align__(16) GsKC {
    uint64_t k;
    double c;
};
__global__ void k_gs_pairs(const uint64_t *keys, const double *coefs, int64_t T, GsKC *out);
template <bool PACKED>
__global__ void k_gs_merge(const uint64_t *keys, const uint32_t *vals, int64_t R, int64_t ta, int64_t tb,
                           const uint64_t *ka, const uint64_t *kb, int raw_bits, const double *ca,
                           const double *cb, const GsKC *pa, const GsKC *pb, double tol, RadixDecode dec,
                           uint64_t *st_key, double *st_coef, int64_t *seg_count, int64_t *stage_off);
__global__ void k_gs_rowptr(const int64_t *out_off, int64_t nblocks, int64_t *row_ptr);

}  // namespace polyhip
