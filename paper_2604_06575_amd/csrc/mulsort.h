// Global radix-sort path of times + simplify for one large pair
// (mulsort.hip): launch constants and kernels.
#pragma once
#include "internal.h"

namespace polyhip {

constexpr int GS_THREADS = 1024;
constexpr int GS_ITEMS = 4;
constexpr int GS_TILE = GS_THREADS * GS_ITEMS;   // elements per workgroup and pass
constexpr int GS_BITS = 8;                       // digit width
constexpr int GS_BINS = 1 << GS_BITS;
constexpr int GS_HIST_THREADS = 256;
constexpr int GS_SORT1_CAP = 8192;               // partner terms sorted by one workgroup
__global__ void k_gs_sort_partner(const uint64_t *keys, const double *coefs, int64_t T, uint64_t *keys_s,
                                  uint32_t *perm, double *coefs_s);
__global__ void k_gs_generate(const uint64_t *ka, const uint64_t *kb_s, int64_t ta, int64_t tb, uint64_t *keys,
                              uint32_t *vals);
__global__ void k_gs_hist(const uint64_t *keys, int64_t R, int shift, int64_t nblocks, int64_t *hist);
__global__ void k_gs_scatter(const uint64_t *keys_in, const uint32_t *vals_in, int64_t R, int shift,
                             int64_t nblocks, const int64_t *hist_off, uint64_t *keys_out, uint32_t *vals_out);
__global__ void k_gs_merge(const uint64_t *keys, const uint32_t *vals, int64_t R, int64_t ta, int64_t tb,
                           const double *ca, const double *cb_s, double tol, uint64_t *st_key, double *st_coef,
                           int64_t *seg_count, int64_t *stage_off);
__global__ void k_gs_rowptr(const int64_t *out_off, int64_t nblocks, int64_t *row_ptr);

}  // namespace polyhip
