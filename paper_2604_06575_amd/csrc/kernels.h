// Kernel declarations shared between the HIP translation units.
#pragma once

#include "internal.h"
#include "mulsort.h"

namespace polyhip {

// Launch parameters set by the autotuner (process-wide; see poly_tune_set).
struct Tunables {
    int64_t mul_bucket_terms;
    int64_t seg_blocks_per_cu;
    int64_t eval_blocks_per_cu;
    int64_t mul_sort_min_raw;
    int64_t simplify_wide_min;
    int64_t deriv_fused_max_n;
    int64_t sort_digit_bits;
    int64_t dense_f64_rows;
};
Tunables tunables();
int sort_bits();
int64_t sort_bins();

// ------------------------------------------------------------ simplify / sort
constexpr int SEG_THREADS = 512;
constexpr int SEG_ITEMS = 8;
constexpr int SEG_CAP = SEG_THREADS * SEG_ITEMS;  // terms held in LDS by one tile

struct SegArgs {
    const int64_t *rp;          // [P+1] CSR of the segments
    const uint64_t *keys;       // packed keys at input positions
    const double *coefs;        // input coefficients (merge mode)
    const int64_t *order;       // [P] processing order (largest first)
    int64_t P;
    unsigned long long *queue;  // job counter, zero before launch
    uint64_t *st_key;           // staging keys, written at input positions
    double *st_coef;            // staging merged coefficients (merge mode)
    uint32_t *st_idx;           // staging local term index (sort-only mode)
    int64_t *seg_count;         // [P] terms written per segment
    double tol;
};

__global__ void k_pack(const uint8_t *__restrict__ exps, int64_t T, int n, int bits, int max_exp,
                       uint64_t *__restrict__ keys, int32_t *status);
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t count);
__global__ void k_order_by_size(const int64_t *rp, int64_t P, int64_t *order);
__global__ void k_seg_merge(SegArgs A);
__global__ void k_seg_sort(SegArgs A);
__global__ void k_seg_sort2(SegArgs A, SegArgs B);
__global__ void k_scan_counts(const int64_t *counts, int64_t S, int64_t *out);
// Single-pass exclusive scan (decoupled look-back).  `state` holds 2 +
// ceil(S / LB_TILE) words that must be zero on entry; they are not on exit.
constexpr int LB_THREADS = 256;
constexpr int LB_ITEMS = 16;
constexpr int64_t LB_TILE = LB_THREADS * LB_ITEMS;
__global__ void k_scan_lookback(const int64_t *in, int64_t S, int64_t *out, unsigned long long *state,
                                int32_t *status);
__global__ void k_compact(const int64_t *stage_off, const int64_t *seg_count, const int64_t *out_off,
                          const uint64_t *st_key, const double *st_coef, int n, int bits,
                          uint8_t *out_exps, double *out_coefs, int64_t capacity, int32_t *status);

// ------------------------------------------------------------------------ mul
constexpr int MUL_THREADS = 256;
constexpr int MUL_CAP = 4096;
constexpr int64_t MUL_TARGET = 3072;       // raw terms per bucket, global-memory bucket kernel
constexpr int64_t MB_TARGET = 32768;       // raw terms per bucket, LDS bucket kernel
constexpr int MUL_SAMPLE = 8192;           // splitter sample per pair
constexpr int64_t MUL_MAX_BUCKETS = 4096;  // per pair

__host__ __device__ inline int64_t mul_buckets_for(int64_t raw, int64_t target)
{
    if (raw <= target) return 1;
    int64_t b = (raw + target - 1) / target;
    return b > MUL_MAX_BUCKETS ? MUL_MAX_BUCKETS : b;
}

struct MulArgs {
    int64_t P;
    const int64_t *a_rp, *b_rp;
    const double *a_c, *b_c;
    const uint64_t *ka, *kb;        // packed keys, storage order
    const uint64_t *ka_s, *kb_s;    // keys sorted per polynomial
    const uint32_t *perm_a, *perm_b;  // local index of each sorted position
    const double *ca_s, *cb_s;      // coefficients in sorted order
    const int64_t *pb_start;        // [P+1] first bucket of each pair
    int32_t *bk_pair;
    uint64_t *bk_lo, *bk_hi;        // inclusive key range of each bucket
    int64_t *bk_stage_off, *bk_count;
    unsigned long long *stage_cursor;
    uint64_t *st_key;
    double *st_coef;
    double tol;
    int64_t nbuckets;               // buckets allocated (host plan)
    int64_t st_capacity;            // staging slots allocated
    int32_t *status;
};

__global__ void k_mul_init_buckets(MulArgs A);
__global__ void k_mul_plan(const int64_t *a_rp, const int64_t *b_rp, int64_t P, int64_t *pb_count, int64_t target);
__global__ void k_mul_splitters(MulArgs A);
__global__ void k_mul_buckets(MulArgs A);
// Cursor-based bucket kernel: partner keys (and row keys) resident in LDS.
constexpr int MB_THREADS = 1024;
constexpr int MB_ITEMS = 4;
constexpr int MB_CAP = MB_THREADS * MB_ITEMS;  // raw terms sorted per piece
constexpr int MB_SAMPLE = 2048;                // sampled raw keys per bucket (piece boundaries)
constexpr int MB_STACK = 112;                  // pending key ranges (pieces + bisection)
constexpr int MB_RPT = 5;                     // rows per thread -> at most 5120 rows
constexpr int MB_MAX_ROWS = MB_THREADS * MB_RPT;
// dynamic LDS of the LDS bucket kernel: the partner keys
__host__ __device__ inline size_t mb_lds_bytes(int64_t ns, int64_t nrows)
{
    (void)nrows;
    return (size_t)ns * 8;
}
constexpr size_t MB_LDS_LIMIT = 72 * 1024;     // with the static part, within 160 KB
constexpr int64_t MB_MAX_PARTNERS = 1 << 30;
__global__ void k_mul_buckets_lds(MulArgs A);
__global__ void k_mul_sorted_coefs(const int64_t *rp, const uint32_t *perm, const double *c, double *out);
__global__ void k_mul_rowptr(const int64_t *out_off, const int64_t *pb_start, int64_t P, int64_t *out_rp,
                             int64_t nbuckets);

// Host-side measurement hook (poly_timing_*): records HIP events on the
// launch stream around a kernel when timing is enabled.
struct TimedLaunch {
    hipEvent_t e1 = nullptr;
    TimedLaunch(int slot, hipStream_t s);
    void done(hipStream_t s);
};

// ---------------------------------------------------------------- derivatives
constexpr int JAC_THREADS = 256;
constexpr int DF_MAX_GROUPS = 256;       // groups (variables or pairs) per formation pass

struct FormArgs {
    const int64_t *rp;          // [P+1] source CSR
    const uint8_t *exps;
    const double *coefs;
    int n;
    int mode;                   // 0: jacobian, 1: hessian entries from a jacobian (group = variable)
    int keep_coefs;             // 1: formed terms keep the source coefficient
    int64_t ngroups;            // n
    const int64_t *item_start;  // [P+1] first work item of each source polynomial
    int64_t P;
    int64_t chunk;              // source terms per work item
    int64_t *cnt;               // per p: [group][chunk] survivor counts
    int64_t *out_rp;            // [P*ngroups + 1]
    uint8_t *out_exps;
    double *out_coefs;
    int64_t capacity;
    int32_t *status;
    int32_t overflow_code;
};

__global__ void k_item_count(const int64_t *rp, int64_t P, int64_t chunk, int64_t *items);
__global__ void k_form_count(FormArgs A);
__global__ void k_form_rowptr(FormArgs A, const int64_t *off);
__global__ void k_form_write(FormArgs A, const int64_t *off);

// ----------------------------------------------------------------- sparse eval
constexpr int EV_WAVES = 8;
constexpr int EV_THREADS = EV_WAVES * kWave;  // 8 waves share 64 points

// OUT_HESS: polynomial q = (p * n + j) * n + k is the Hessian entry (j, k) of f_p, written (k >= j) to a
// point-contiguous staging row Y[q * N + pt] that k_hess_transpose turns into both triangles
enum OutMode { OUT_EVAL = 0, OUT_GRAD = 1, OUT_HESS = 2 };

struct EvalArgs {
    const int64_t *rp;            // [Q+1]
    const uint8_t *exps;          // [T * n] exponent rows
    const double *coefs;          // [T]
    int n;
    const double *X;              // [N * n]
    int64_t N;
    int64_t Q;                    // polynomials
    int mode;                     // OutMode
    double *Y;                    // output
    int64_t term_limit;           // terms at or beyond this index are never read
    const uint32_t *maxdeg;       // bound on every term's degree (2, 3, 4; else 255), recorded by k_encode_factors, or null
};

__global__ void k_encode_support(const uint8_t *exps, int64_t T, int n, uint64_t *enc, const int64_t *used);
constexpr int EV_MAX_DEG = 12;   // total degree handled by the factor-list encoding
// maxdeg (or null): a zeroed word that receives, by atomicMax, the largest
// degree class of the encoded terms (2 for degree <= 2, then 3, 4, and 255)
__global__ void k_encode_factors(const uint8_t *exps, int64_t T, int n, uint32_t *enc, const int64_t *used,
                                 uint32_t *maxdeg);

// products of polynomial matrices (matrix.hip)
constexpr int MAT_THREADS = 256;
__global__ void k_mat_raw_sizes(const int64_t *a_rp, const int64_t *b_rp, int64_t I, int64_t K, int64_t J,
                                int64_t *sizes);
__global__ void k_mat_expand(const int64_t *a_rp, const uint8_t *a_e, const double *a_c, const int64_t *b_rp,
                             const uint8_t *b_e, const double *b_c, int64_t I, int64_t K, int64_t J, int n,
                             const int64_t *r_rp, uint8_t *r_e, double *r_c);
__global__ void k_mat_keys(const int64_t *a_rp, const uint64_t *ka, const double *a_c, const int64_t *b_rp,
                           const uint64_t *kb, const double *b_c, int64_t I, int64_t K, int64_t J,
                           const int64_t *r_rp, int64_t R, uint64_t span, uint64_t *keys, uint32_t *vals,
                           double *r_c);

__global__ void k_concat_copy(const int64_t *rp, const uint8_t *exps, const double *coefs, int64_t P, int64_t T,
                              int n, int64_t entry_off, int64_t term_off, int64_t *out_rp, uint8_t *out_exps,
                              double *out_coefs);

// device-wide simplify of batches with large polynomials (wide.hip)
__global__ void k_ws_keys(const uint8_t *exps, int64_t T, int n, uint32_t radix, int max_exp,
                          const int64_t *row_ptr, int64_t P, uint64_t span, uint64_t *keys, uint32_t *vals,
                          int32_t *status);
__global__ void k_ws_merge(const uint64_t *keys, const uint32_t *vals, int64_t R, const double *coefs, double tol,
                           uint64_t span, uint32_t radix, int n, int bits, uint64_t *st_key, uint64_t *st_ckey,
                           double *st_coef, int64_t *seg_count, int64_t *stage_off);
__global__ void k_ww_word(const uint8_t *exps, int64_t T, int n, uint32_t radix, int max_exp, int lo, int hi,
                          int with_poly, const int64_t *row_ptr, int64_t P, uint64_t *keys, int32_t *status);
__global__ void k_ww_gather(const uint64_t *src, const uint32_t *vals, int64_t R, uint64_t *dst);
__global__ void k_ww_iota(uint32_t *vals, int64_t T);
__global__ void k_ww_heads(const uint64_t *keys, const uint32_t *vals, int64_t R, const uint8_t *exps, int n, int lo,
                           uint8_t *head);
__global__ void k_ww_merge(const uint64_t *keys, const uint32_t *vals, const uint8_t *head, int64_t R,
                           const double *coefs, double tol, uint32_t *st_idx, uint64_t *st_ckey, double *st_coef,
                           int64_t *seg_count, int64_t *stage_off, const uint64_t *low, uint64_t *st_low);
__global__ void k_ww_word2(const uint8_t *exps, int64_t T, int n, uint32_t radix, int max_exp, int lo0, int hi0,
                           int lo1, int hi1, int with_poly, const int64_t *row_ptr, int64_t P, uint64_t *keys0,
                           uint64_t *copy0, uint64_t *keys1, int32_t *status);
__global__ void k_ww_heads2(const uint64_t *top, const uint64_t *low, int64_t R, uint8_t *head);
__global__ void k_ww_compact2(const int64_t *stage_off, const int64_t *seg_count, const int64_t *out_off,
                              const uint64_t *st_top, const uint64_t *st_low, const double *st_coef, int n, int split,
                              uint64_t radix, int chunk, uint64_t div, uint64_t div_magic, uint32_t digit_magic,
                              uint8_t *out_exps, double *out_coefs, int64_t capacity, int32_t *status);
__global__ void k_ww_compact(const int64_t *stage_off, const int64_t *seg_count, const int64_t *out_off,
                             const uint32_t *st_idx, const double *st_coef, const uint8_t *exps, int n,
                             uint8_t *out_exps, double *out_coefs, int64_t capacity, int32_t *status);
__global__ void k_mul_raw_sizes(const int64_t *a_rp, const int64_t *b_rp, int64_t P, int64_t *sizes);
__global__ void k_mul_expand_rows(const int64_t *a_rp, const uint8_t *a_e, const double *a_c, int a_max,
                                  const int64_t *b_rp, const uint8_t *b_e, const double *b_c, int b_max, int64_t P,
                                  int n, const int64_t *r_rp, int64_t R, uint8_t *r_e, double *r_c, int32_t *status);
__global__ void k_ws_rowptr(int64_t P, uint64_t span, const uint64_t *keys, int64_t R, const int64_t *stage_off,
                            const int64_t *seg_count, const int64_t *out_off, int64_t nb, const uint64_t *st_ckey,
                            int64_t *row_ptr);

// affine-normal direction (affine.hip): one workgroup per point
constexpr int AN_THREADS = 256;
constexpr int AN_MAX_N = 255;       // every nvars the batches allow
constexpr int AN_MAX_N_LDS = 128;   // largest n whose n x (n+1) matrix is kept in LDS
__host__ __device__ constexpr size_t affine_lds_bytes(int n)
{
    return ((n <= AN_MAX_N_LDS ? (size_t)n * (n + 1) : 0) + 8 * (size_t)n + (size_t)n * (EV_MAX_DEG + 1)) *
           sizeof(double);
}
__global__ void k_affine_normal(int n, const uint4 *enc, const double *coefs, int64_t T, const double *X,
                                const double *G, double *H, double reg, double *D, double *gnorm,
                                int32_t *status);
// affine-normal direction, stochastic route (stochastic.hip): one workgroup
// per point, probes solved AS slots at a time
constexpr int AS_THREADS = 256;
constexpr int AS_MAX_SLOTS = 64;
constexpr size_t AS_LDS_BUDGET = 64 * 1024;
__host__ __device__ constexpr size_t affine_stochastic_lds_bytes(int n, int slots)
{
    return (size_t)(4 + 5 * slots) * n * sizeof(double);
}
struct AffStochArgs {
    int n;
    const uint4 *enc;       // factor lists [T]
    const double *coefs;    // [T]
    int64_t T;
    const double *X;        // [N][n]
    const double *Z;        // probes [q][n], or [N][q][n] when per_point
    int per_point;
    int q;
    int slots;              // probes solved at once, a power of two <= AS_MAX_SLOTS
    double reg, tol;
    int maxit;
    double *D;              // [N][n]
    double *gnorm;          // [N]
    int32_t *hv;            // [N] or null
    int32_t *status;
};
__global__ void k_affine_stochastic(AffStochArgs A);
__global__ void k_eval_terms(EvalArgs A, const uint32_t *enc, double *partial, int64_t S);
// k_eval_terms for batches whose recorded degree class (A.maxdeg) is at most
// 4; each of the two returns at once where the other applies
__global__ void k_eval_terms_short(EvalArgs A, const uint32_t *__restrict__ enc, const double *__restrict__ coefs,
                                   double *partial, int64_t S);
__global__ void k_eval_reduce(EvalArgs A, const double *partial, int64_t S);
__global__ void k_hess_transpose(const double *stage, int64_t P, int64_t N, int n, double *H);
// CSR batches over a shared basis (dense.hip)
__global__ void k_check_shared(const uint8_t *exps, int64_t P, int64_t K, int n, int32_t *status);
__global__ void k_derive_basis(const uint8_t *basis, int64_t K, int n, int j, int k, uint8_t *dbasis, const double *C,
                               int64_t P, double *dC);
__global__ void k_hess_mirror(double *H, int64_t PN, int n);
__global__ void k_eval_wsum(EvalArgs A, const uint32_t *enc, const double *gY, int64_t P, int64_t S, double *out,
                            double *partial);
__global__ void k_eval_wsum_short(EvalArgs A, const uint32_t *__restrict__ enc, const double *__restrict__ coefs,
                                  const double *gY, int64_t P, int64_t S, double *out, double *partial);
constexpr int64_t EV_TARGET_WAVES = 16384;   // waves wanted before polynomials are cut into segments
constexpr int64_t EV_MIN_SEGMENT = 32;       // fewest terms per segment
constexpr int64_t EV_MAX_SEGMENTS = 256;


// fused derivative streaming (deriv.hip)
enum DerivMode { DM_GRAD = 0, DM_DX = 1, DM_HVP = 2, DM_DIRD = 3 };
struct DerivArgs {
    const int64_t *rp;        // [P+1] source CSR
    int64_t P;
    int64_t T;                // terms (rp[P])
    const uint8_t *exps;      // [T * n] (terms with more than eight variables read their dense row)
    const double *coefs;      // c
    const double *coefs2;     // w (DM_HVP, DM_DIRD), may be null
    const uint64_t *enc;      // support encoding (k_encode_support), two words per term
    int n;
    const double *X;          // [N * n]
    int64_t N;
    const double *gY;         // [P * N] (DM_DX, DM_HVP)
    const double *U;          // [N * n] direction (DM_HVP, DM_DIRD), may be null for DM_DIRD
    int64_t S;                // term segments per unit
    double *out;
    double *partial;          // S > 1: S slices in the output layout
};
template <int MODE>
__global__ void k_deriv_terms(DerivArgs A);
__global__ void k_sum_slices(const double *partial, int64_t L, int64_t S, double *out);
__global__ void k_backward2_dc(const int64_t *rp, int64_t P, const uint8_t *exps, int n, int64_t T, const double *X,
                               const double *U, int64_t N, const double *gY, double *partial, const uint64_t *enc,
                               int cp);
constexpr int DV_ACC_PITCH = 65;                 // doubles per accumulator row (64 points + 1)
constexpr size_t DV_LDS_MAX = 160 * 1024;        // LDS of one workgroup on gfx950
constexpr int BWC_THREADS = 256;
constexpr int BWC_POINTS = 512;   // points per chunk
constexpr int BWC_TERMS = 4;      // terms per thread
__global__ void k_backward_dc(const int64_t *rp, int64_t P, const uint8_t *exps, int n, int64_t T, const double *X,
                              int64_t N, const double *gY, double *partial, int64_t nchunks,
                              const uint4 *fenc, int cp);
__global__ void k_backward_dc_reduce(const double *partial, int64_t T, int64_t nchunks, double *dC);

}  // namespace polyhip
