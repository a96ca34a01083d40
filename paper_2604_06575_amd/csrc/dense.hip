// Evaluation of P polynomials over one shared monomial set: Y = C V with
// C [P x K] the coefficient matrix and V [K x N] the monomial values
// V[k][pt] = prod_i x_pt,i ^ e_k,i (Section 3.3 eval, applied to a polynomial
// matrix whose entries share a basis as produced by monolist, Section 3.1).
// This is the one dense contraction of the path, so it runs on MFMA.  V is
// never stored: each workgroup builds its K-slice of V from the points'
// coordinates in LDS.
//
// FP64 path: v_mfma_f64_16x16x4f64, FP64 V.
//
// Split path (error-free splitting in the style of Ozaki, Ogita, Oishi and
// Rump): within each K-block of 128 monomials every row of C and every
// column of V gets a power-of-two scale 2^sigma above its largest magnitude.
// Each value x is cut into S integer digits m_1..m_S (|m_1| <= 256,
// |m_s| <= 128 after), x = sum_s m_s 2^(sigma - 8 s) + r, |r| <= 2^(sigma - 8S - 1).
// A digit carried with its scale is an exact BF16 number.  Digit products of
// one diagonal d = s + t share the scale 2^(sigma_C + sigma_V - 8d), and their
// integer sum over a K-block stays below 2^24, so BF16 MFMA with FP32
// accumulation adds them exactly; each diagonal's FP32 sum is moved to an
// FP64 accumulator after every K-block.  Pairs with s + t > S + 1 are
// dropped; the result's error relative to sum_k |C v| is about 2^-(8S-10).
#include <string.h>

#include <algorithm>

#include "kernels.h"

namespace polyhip {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int DN_KB = 128;      // K-block of the split scheme (exact FP32 sums)

// ---------------------------------------------------------------- helpers

__device__ inline double powi_d(double x, uint32_t e)
{
    double p = x;
    for (uint32_t k = 1; k < e; ++k) p = p * x;
    return p;
}

// Monomial value of a basis term from its factor list (k_encode_factors
// layout: up to EV_MAX_DEG variable indices, padded with n, degree in the
// last word) at the point x[i * xs], i = variable; the point tile holds a row
// of ones at i = n.  The reads of a chunk of four factors are issued before
// its multiplications; the product runs left to right.  Terms of higher
// degree are evaluated from their exponent row.
__device__ inline double factor_chunk(double v, uint32_t word, const double *x, int xs)
{
    const double x0 = x[(word & 0xffu) * xs];
    const double x1 = x[((word >> 8) & 0xffu) * xs];
    const double x2 = x[((word >> 16) & 0xffu) * xs];
    const double x3 = x[(word >> 24) * xs];
    return (((v * x0) * x1) * x2) * x3;
}

__device__ inline double factor_value(const uint4 &w, const uint8_t *row, int n, const double *x, int xs)
{
    const uint32_t d = w.w;
    double v = 1.0;
    if (d > (uint32_t)EV_MAX_DEG) {
        for (int i = 0; i < n; ++i)
            if (row[i]) v = v * powi_d(x[i * xs], row[i]);
        return v;
    }
    if (d > 0) v = factor_chunk(v, w.x, x, xs);
    if (d > 4) v = factor_chunk(v, w.y, x, xs);
    if (d > 8) v = factor_chunk(v, w.z, x, xs);
    return v;
}

// exponent sigma with |x| < 2^sigma for the largest |x| of a block (x = 0 -> -1100)
__device__ inline int scale_exp(double amax)
{
    if (!(amax > 0.0)) return -1100;
    int e;
    (void)frexp(amax, &e);
    return e;
}

__device__ inline unsigned short bf16_bits_exact(float f)
{
    return (unsigned short)(__float_as_uint(f) >> 16);
}

// ------------------------------------------------------------ FP64 kernel

constexpr int D64_BN = 128, D64_KS = 16, D64_THREADS = 256;   // rows per workgroup: BM, 64 or 128

// grid: x = N tiles (fastest, so concurrently running workgroups share a C
// row panel), y = P tiles of BM rows (64 or 128: each wave holds BM / 32
// row tiles of 16 against four column tiles, so a V tile formed in LDS feeds
// BM rows).  Dynamic LDS: (n + 1) * D64_BN doubles for the
// points and a row of ones.  Each K step: the C tile and the factor lists of
// the step after next are loaded into registers (buffer loads, so the only
// per-thread addresses are 32-bit offsets and no load waits on another),
// the MFMAs of this step run, and the V tile of the next step is formed from
// factor lists staged in LDS one step ahead.
template <int BM>
__global__ void __launch_bounds__(D64_THREADS) k_dense_f64(int n, int64_t K, const uint8_t *basis,
                                                           const uint4 *enc, int64_t P, const double *C,
                                                           int64_t N, const double *X, double *Y, int64_t ys)
{
    constexpr int RT = BM / 32;                        // 16-row MFMA tiles per wave
    constexpr int TPR = D64_THREADS / BM, CPT = D64_KS / TPR;   // C tile loads: threads per row, entries per thread
    extern __shared__ double s_x[];                    // [n + 1][D64_BN], last row ones
    __shared__ double s_c[BM][D64_KS + 1];
    __shared__ double s_v[D64_KS][D64_BN + 2];
    __shared__ uint4 s_enc[2][D64_KS];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;                 // wave: BM / 2 rows x 64 points
    const int64_t r0 = (int64_t)blockIdx.y * BM;
    const int64_t n0 = (int64_t)blockIdx.x * D64_BN;
    for (int idx = tid; idx < (n + 1) * D64_BN; idx += D64_THREADS) {
        const int i = idx / D64_BN, c = idx % D64_BN;
        const int64_t pt = n0 + c;
        s_x[idx] = i == n ? 1.0 : (pt < N ? X[pt * n + i] : 0.0);
    }
    d4v acc[RT][4];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
    // load roles: C tile row/k of this thread, V tile point/k of this thread
    const int crow = tid / TPR, ckk = (tid % TPR) * CPT;
    const int vcol = tid & (D64_BN - 1), vkb = (tid >> 7) * 8;
    // this block's rows of C as one buffer: rows past P read as zero; the
    // host keeps BM * K * 8 bytes below 2^31
    const int rows_here = (int)(P - r0 < BM ? P - r0 : BM);
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)(C + r0 * K), (short)0,
                                                                       rows_here * (int)K * 8, 0x00020000);
    const int cbase = (crow * (int)K + ckk) * 8;
    double creg[CPT], vreg[8];
    uint4 ereg = make_uint4(0, 0, 0, 0);
    auto load_c = [&](int64_t kk) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)   // entries past K (next row's) are masked when stored
            creg[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, cbase + ((int)kk + q) * 8, 0, 0));
    };
    auto load_enc = [&](int64_t kk) {   // factor lists of k = kk + tid, tid < D64_KS (zero past K)
        if (tid < D64_KS) {
            const __amdgpu_buffer_rsrc_t re = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(enc + kk), (short)0, (int)((K - kk) * 16 > 0 ? (K - kk) * 16 : 0), 0x00020000);
            const u32x4 e = __builtin_amdgcn_raw_buffer_load_b128(re, tid * 16, 0, 0);
            ereg = make_uint4(e[0], e[1], e[2], e[3]);
        }
    };
    auto form_v = [&](int64_t kk, const uint4 *le) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            vreg[q] = kk + vkb + q < K ? factor_value(le[vkb + q], basis + (kk + vkb + q) * n, n, s_x + vcol, D64_BN)
                                       : 0.0;
    };
    // stage 0 operands; factor lists of step 1 in flight
    load_enc(0);
    load_c(0);
    __syncthreads();
    if (tid < D64_KS) s_enc[0][tid] = ereg;
    load_enc(D64_KS);
    __syncthreads();
    form_v(0, s_enc[0]);
    int par = 1;   // s_enc buffer of the next step's factor lists
    for (int64_t k0 = 0; k0 < K; k0 += D64_KS) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CPT; ++q) s_c[crow][ckk + q] = k0 + ckk + q < K ? creg[q] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s_v[vkb + q][vcol] = vreg[q];
        if (tid < D64_KS) s_enc[par][tid] = ereg;
        __syncthreads();
        const int64_t k1 = k0 + D64_KS;
        // next stage's C tile and the factor lists after it: in flight while the MFMAs run
        if (k1 < K) {
            load_c(k1);
            load_enc(k1 + D64_KS);
        }
#pragma unroll
        for (int k4 = 0; k4 < D64_KS; k4 += 4) {
            double a[RT], b[4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = s_c[wr * (BM / 2) + rt * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) b[ct] = s_v[k4 + (lane >> 4)][wc * 64 + ct * 16 + (lane & 15)];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], b[ct], acc[rt][ct], 0, 0, 0);
        }
        // next stage's V tile (VALU work beside the MFMAs)
        if (k1 < K) form_v(k1, s_enc[par]);
        par ^= 1;
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // v_mfma_f64_16x16x4f64 result: lane l, register v holds
                // row (l / 16) + 4 v, column l % 16 of the 16 x 16 tile
                const int64_t r = r0 + wr * (BM / 2) + rt * 16 + (lane >> 4) + 4 * v;
                const int64_t c = n0 + wc * 64 + ct * 16 + (lane & 15);
                if (r < P && c < N) Y[(r * N + c) * ys] = acc[rt][ct][v];
            }
}

// ------------------------------------------------------- FP64 reverse mode
//
// Reverse mode of Y = C V for a cotangent gY [P x N]:
//   dC = gY V^T            [P x K]: MFMA over points, V^T built per step
//   dX[pt][j] = sum_k W[k][pt] d v_k / d x_j (x_pt),   W = C^T gY [K x N]
// dX never stores W: a workgroup owns a tile of points, forms W for one
// tile of monomials at a time on MFMA (contraction over the polynomials),
// and contracts it at once with the monomials' first derivatives.

constexpr int DB_BM = 64, DB_BN = 128, DB_KS = 16, DB_THREADS = 256;

// dC tile: rows p (64), columns k (128), contraction over points in steps
// of 16.  Each thread owns one monomial column (its factor list held in
// registers) and forms 8 of its values per step from the step's points,
// staged in LDS (dynamic: (n + 1) * 16 doubles, last row ones).
template <int BM>
__global__ void __launch_bounds__(DB_THREADS) k_dense_bwd_dc(int n, int64_t K, const uint8_t *basis, const uint4 *enc,
                                                            int64_t P, const double *gY, int64_t N, const double *X,
                                                            double *dC)
{
    constexpr int RT = BM / 32;                      // 16-row MFMA tiles per wave
    constexpr int TPR = DB_THREADS / BM, CPT = DB_KS / TPR;   // gY tile loads: threads per row, points per thread
    extern __shared__ double s_xp[];                 // [n + 1][DB_KS]
    __shared__ double s_a[BM][DB_KS + 1];
    __shared__ double s_b[DB_KS][DB_BN + 2];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t r0 = (int64_t)blockIdx.y * BM;
    const int64_t k0 = (int64_t)blockIdx.x * DB_BN;
    const int vcol = tid & (DB_BN - 1), vpb = (tid >> 7) * 8;
    const int64_t kcol = k0 + vcol;
    const uint4 my_enc = kcol < K ? enc[kcol] : make_uint4(0, 0, 0, 0);
    const int arow = tid / TPR, acol = (tid % TPR) * CPT;
    d4v acc[RT][4];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
    for (int64_t p0 = 0; p0 < N; p0 += DB_KS) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int64_t r = r0 + arow, pt = p0 + acol + q;
            s_a[arow][acol + q] = (r < P && pt < N) ? gY[r * N + pt] : 0.0;
        }
        for (int idx = tid; idx < (n + 1) * DB_KS; idx += DB_THREADS) {
            const int i = idx / DB_KS, l = idx % DB_KS;
            const int64_t pt = p0 + l;
            s_xp[idx] = i == n ? 1.0 : (pt < N ? X[pt * n + i] : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q)
            s_b[vpb + q][vcol] =
                kcol < K ? factor_value(my_enc, basis + kcol * n, n, s_xp + vpb + q, DB_KS) : 0.0;
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < DB_KS; k4 += 4) {
            double a[RT], b[4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = s_a[wr * (BM / 2) + rt * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) b[ct] = s_b[k4 + (lane >> 4)][wc * 64 + ct * 16 + (lane & 15)];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], b[ct], acc[rt][ct], 0, 0, 0);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = r0 + wr * (BM / 2) + rt * 16 + (lane >> 4) + 4 * v;
                const int64_t c = k0 + wc * 64 + ct * 16 + (lane & 15);
                if (r < P && c < K) dC[r * K + c] = acc[rt][ct][v];
            }
}

// d v / d x_j for every variable j of a monomial given by its support
// encoding (up to eight (variable, exponent) slots; 0xFFFF: the dense row),
// each added, times w, to acc[j * 64] (an LDS accumulator column).
__device__ inline void add_monomial_grad(const uint64_t w0, const uint64_t w1, const uint8_t *row, int n,
                                         const double *x, int xs, double w, double *acc)
{
    if ((w0 & 0xffffull) == 0xffffull) {
        for (int j = 0; j < n; ++j) {
            const int ej = row[j];
            if (!ej) continue;
            double p = (double)ej;
            for (int i = 0; i < n; ++i) {
                const int ei = row[i] - (i == j);
                if (ei > 0) p = p * powi_d(x[i * xs], (uint32_t)ei);
            }
            __hip_atomic_fetch_add(acc + j * kWave, w * p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        return;
    }
    int var[8], ex[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const uint32_t ent = (uint32_t)(((s < 4 ? w0 : w1) >> (16 * (s & 3))) & 0xffffu);
        var[s] = (int)(ent & 0xffu);
        ex[s] = (int)(ent >> 8);
    }
    double pw[8], pm[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const double xv = x[var[s] * xs];
        double q = 1.0;
        for (int i = 1; i < ex[s]; ++i) q = q * xv;
        pm[s] = q;
        pw[s] = ex[s] ? q * xv : 1.0;
    }
    double pre[9], suf[9];
    pre[0] = 1.0;
    suf[8] = 1.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) pre[s + 1] = pre[s] * pw[s];
#pragma unroll
    for (int s = 7; s >= 0; --s) suf[s] = pw[s] * suf[s + 1];
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (ex[s])
            __hip_atomic_fetch_add(acc + var[s] * kWave, w * ((double)ex[s] * ((pm[s] * pre[s]) * suf[s + 1])),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// dX for one tile of 128 points.  Per monomial tile (64): W tile on MFMA
// (A = C^T rows k, B = gY rows p, contraction over P in steps of 16), then
// each lane's W entries times the derivatives of their monomials at their
// points, added into its wave's accumulator block [n][64 points] (LDS adds:
// one wave's adds apply in program and lane order, so the sums do not
// depend on scheduling).  The two waves covering the same points are added
// in a fixed order at the end.  Dynamic LDS: points [(n + 1)][128] and four
// accumulator blocks [n][64].
__global__ void __launch_bounds__(DB_THREADS) k_dense_bwd_dx(int n, int64_t K, const uint8_t *basis,
                                                            const uint64_t *senc, int64_t P, const double *C,
                                                            const double *gY, int64_t N, const double *X, double *dX)
{
    extern __shared__ double s_dyn[];
    double *s_x = s_dyn;                                    // [n + 1][DB_BN]
    double *s_acc = s_dyn + (size_t)(n + 1) * DB_BN;        // [4][n][64]
    __shared__ double s_a[DB_BM][DB_KS + 1];                // C^T tile: [k][p]
    __shared__ double s_b[DB_KS][DB_BN + 2];                // gY tile: [p][pt]
    __shared__ uint64_t s_enc[DB_BM][2];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t n0 = (int64_t)blockIdx.x * DB_BN;
    for (int idx = tid; idx < (n + 1) * DB_BN; idx += DB_THREADS) {
        const int i = idx / DB_BN, c = idx % DB_BN;
        const int64_t pt = n0 + c;
        s_x[idx] = i == n ? 1.0 : (pt < N ? X[pt * n + i] : 0.0);
    }
    for (int idx = tid; idx < 4 * n * kWave; idx += DB_THREADS) s_acc[idx] = 0.0;
    double *my_acc = s_acc + (size_t)w * n * kWave;
    for (int64_t k0 = 0; k0 < K; k0 += DB_BM) {
        __syncthreads();
        if (tid < DB_BM) {
            const int64_t k = k0 + tid;
            s_enc[tid][0] = k < K ? senc[2 * k] : 0ull;
            s_enc[tid][1] = k < K ? senc[2 * k + 1] : 0ull;
        }
        d4v acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
        // operand tiles of a step: C^T (16 polynomials x 64 monomials, read
        // along k) and gY (16 polynomials x 128 points, read along the points);
        // the next step's are loaded into registers while this step's MFMAs run
        double ra[4], rb[8];
        auto load_tiles = [&](int64_t p0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = tid + q * DB_THREADS;
                const int pp = idx / DB_BM, kr = idx % DB_BM;
                const int64_t p = p0 + pp, k = k0 + kr;
                ra[q] = (p < P && k < K) ? C[p * K + k] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int idx = tid + q * DB_THREADS;
                const int pp = idx / DB_BN, c = idx % DB_BN;
                const int64_t p = p0 + pp, pt = n0 + c;
                rb[q] = (p < P && pt < N) ? gY[p * N + pt] : 0.0;
            }
        };
        load_tiles(0);
        for (int64_t p0 = 0; p0 < P; p0 += DB_KS) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = tid + q * DB_THREADS;
                s_a[idx % DB_BM][idx / DB_BM] = ra[q];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int idx = tid + q * DB_THREADS;
                s_b[idx / DB_BN][idx % DB_BN] = rb[q];
            }
            __syncthreads();
            if (p0 + DB_KS < P) load_tiles(p0 + DB_KS);
#pragma unroll
            for (int k4 = 0; k4 < DB_KS; k4 += 4) {
                double a[2], b[4];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) a[rt] = s_a[wr * 32 + rt * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) b[ct] = s_b[k4 + (lane >> 4)][wc * 64 + ct * 16 + (lane & 15)];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], b[ct], acc[rt][ct], 0, 0, 0);
            }
        }
        // W tile entries times the monomials' derivatives at their points
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kr = wr * 32 + rt * 16 + (lane >> 4) + 4 * v;
                const int64_t k = k0 + kr;
                if (k >= K) continue;
                const uint64_t e0 = s_enc[kr][0], e1 = s_enc[kr][1];
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int pl = ct * 16 + (lane & 15);   // point within the wave's 64
                    add_monomial_grad(e0, e1, basis + k * n, n, s_x + wc * 64 + pl, DB_BN, acc[rt][ct][v],
                                      my_acc + pl);
                }
            }
    }
    __syncthreads();
    // waves (0, wc) and (1, wc) cover the same 64 points: add in that order
    for (int idx = tid; idx < DB_BN * n; idx += DB_THREADS) {
        const int pl = idx / n, j = idx % n;
        const int c = pl >> 6, l = pl & 63;
        const int64_t pt = n0 + pl;
        if (pt < N)
            dX[pt * n + j] = s_acc[((size_t)(0 * 2 + c) * n + j) * kWave + l] +
                             s_acc[((size_t)(1 * 2 + c) * n + j) * kWave + l];
    }
}

// ------------------------------------------------------------ split kernels

// BF16 digit planes of C with their scale folded in, stored in the operand
// order of the 32 x 32 x 16 BF16 MFMA: plane s, row block rb = r / 32, k
// chunk kc = k / 16 form one 1 KB record in which lane l = r % 32 + 32 *
// ((k % 16) / 8) holds k % 8 = 0..7 as 16 contiguous bytes.  Rows are padded
// to a multiple of 32 and k to Kp (multiple of SP_KS) with zero digits, so a
// wave loads its A operand as one coalesced 1 KB read.  One block per (row,
// K-block): thread k of the block owns column k0 + k.
__host__ __device__ inline int64_t split_c_index(int64_t s, int64_t r, int64_t k, int64_t RB, int64_t Kp)
{
    const int64_t lane = (r & 31) + 32 * ((k & 15) >> 3);
    return ((((s * RB + (r >> 5)) * (Kp >> 4) + (k >> 4)) * 64 + lane) << 3) + (k & 7);
}

__global__ void __launch_bounds__(DN_KB) k_split_c(const double *C, int64_t P, int64_t K, int64_t Kp, int S,
                                                   unsigned short *Cs)
{
    __shared__ double s_red[DN_KB / kWave];
    const int64_t nkb = ceil_div(Kp, DN_KB);
    const int64_t RB = ceil_div(P, 32);
    const int64_t r = blockIdx.x / nkb, kb = blockIdx.x % nkb;
    const int64_t k = kb * DN_KB + threadIdx.x;
    const double x = (r < P && k < K) ? C[r * K + k] : 0.0;
    double a = fabs(x);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, kWave));
    if (lane_id() == 0) s_red[threadIdx.x >> 6] = a;
    __syncthreads();
    double amax = s_red[0];
#pragma unroll
    for (int i = 1; i < DN_KB / kWave; ++i) amax = fmax(amax, s_red[i]);
    if (k >= Kp) return;
    const int sig = scale_exp(amax);
    double y = amax > 0.0 ? ldexp(x, -sig) : 0.0;
    for (int s = 1; s <= S; ++s) {
        y = y * 256.0;
        const double m = rint(y);
        y = y - m;
        Cs[split_c_index(s - 1, r, k, RB, Kp)] = bf16_bits_exact(ldexpf((float)m, sig - 8 * s));
    }
}

// Column scales of V per K-block: sig_v[kb * N + pt].  One block per
// (K-block, 64 points); thread (point, group) scans 32 monomials.
__global__ void __launch_bounds__(256) k_split_vscale(int n, int64_t K, const uint8_t *basis, const uint4 *enc,
                                                      int64_t N, const double *X, int32_t *sig_v)
{
    extern __shared__ double s_xv[];               // [n + 1][64], last row ones
    __shared__ double s_m[4][64];
    const int64_t ntile = ceil_div(N, 64);
    const int64_t kb = blockIdx.x / ntile, pt0 = (blockIdx.x % ntile) * 64;
    for (int idx = threadIdx.x; idx < (n + 1) * 64; idx += 256) {
        const int i = idx / 64, c = idx % 64;
        s_xv[idx] = i == n ? 1.0 : (pt0 + c < N ? X[(pt0 + c) * n + i] : 0.0);
    }
    __syncthreads();
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    double amax = 0.0;
    for (int q = 0; q < DN_KB / 4; ++q) {
        const int64_t k = kb * DN_KB + g * (DN_KB / 4) + q;
        if (k < K) amax = fmax(amax, fabs(factor_value(enc[k], basis + k * n, n, s_xv + c, 64)));
    }
    s_m[g][c] = amax;
    __syncthreads();
    if (g == 0 && pt0 + c < N)
        sig_v[kb * N + pt0 + c] = scale_exp(fmax(fmax(s_m[0][c], s_m[1][c]), fmax(s_m[2][c], s_m[3][c])));
}

// The S digits of y (|y| < 1), each times its scale (an exact BF16
// number), into BF16 slot q of a thread's packed digit words dig[d][q / 2].
// y is taken to 48 bits as yh + yl and the digits are extracted in FP32.
template <int S>
__device__ inline void put_digits(double y, const float *scale, int q, uint32_t (*dig)[2])
{
    const float yh = (float)y;
    const float yl = (float)(y - (double)yh);
    float t = yh;
    float m[S];
#pragma unroll
    for (int d = 0; d < S; ++d) {
        if (d == 3) t = t + yl * 16777216.0f;   // yl in the frame of digit 4
        t = t * 256.0f;
        m[d] = rintf(t);
        t = t - m[d];
    }
#pragma unroll
    for (int d = 0; d < S; ++d) {
        const float f = m[d] * scale[d];
        if (q & 1) dig[d][q >> 1] = (dig[d][q >> 1] & 0xffffu) | (__float_as_uint(f) & 0xffff0000u);
        else dig[d][q >> 1] = __float_as_uint(f) >> 16;
    }
}

constexpr int SP_KS = 32, SP_THREADS = 512;
constexpr int SP_BM = 256, SP_BN = 64;   // workgroup tile: 8 waves x (32 rows x 64 points)
// FP32 accumulator groups per tile: diagonals 2 and 3 (exact integer sums on
// their own scale) and one shared group for diagonals >= 4 (at most 2^-16 of
// the leading term), whose FP32 rounding sets an error floor near 2^-34 of
// sum |C v| per K-block whatever the digit count; a fourth exact group would
// lower it but does not fit the register budget of this tile shape, so no
// more than five digits are offered (a sixth would sit below that floor).
constexpr int SP_GROUPS = 3;
constexpr int SP_LDK = SP_KS + 8;    // padded k stride (bf16 elements) of the LDS digit planes
constexpr int SP_VK = SP_KS * SP_BN / SP_THREADS;   // V values per thread per K step

__host__ __device__ constexpr size_t split_lds_bytes(int n, int S)
{
    return (size_t)SP_THREADS * 16 * 8 + (size_t)(n + 1) * SP_BN * 8 + (size_t)2 * S * SP_BN * SP_LDK * 2 +
           (size_t)2 * SP_KS * 16;
}

// grid: x = N tiles of SP_BN, y = P tiles of SP_BM.  Wave w owns rows
// r0 + 32 w .. + 31 and all SP_BN points (two 32 x 32 MFMA tiles, SP_GROUPS
// accumulator groups each).  Its C digits arrive straight from the
// MFMA-ordered planes into registers (buffer loads, issued as soon as the
// step's MFMAs have consumed the previous ones); the V digits of a K step are
// formed once per workgroup into LDS and feed all 8 waves.  V digits and the
// step's factor lists are double-buffered, so a K step needs one barrier, and
// the MFMAs of step i and the digit formation of step i + 1 sit in one
// straight-line block: the formation assumes degree <= 4 (one factor word,
// no branches), so its VALU and LDS work can issue between the MFMAs; a
// thread whose monomials have higher degree redoes its values afterwards.
// The FP64 sums of the first MFMA tile stay in registers, those of the second
// in LDS (register budget of two waves per SIMD).  Dynamic LDS: FP64 sums
// [8 waves][16][64 lanes], points [n + 1][BN] doubles (last row ones), V
// digits [2][S][BN][SP_LDK] bf16, factor lists [2][SP_KS].
template <int S>
__global__ void __launch_bounds__(SP_THREADS) k_dense_split(int n, int64_t K, int64_t Kp, const uint8_t *basis,
                                                            const uint4 *enc, int64_t P,
                                                            const unsigned short *Cs, int64_t N, const double *X,
                                                            const int32_t *sig_v, double *Y, int64_t ys)
{
    static_assert(SP_VK == 4, "V digits are stored as 2 words per plane");
    extern __shared__ double s_dyn[];
    double *s_out = s_dyn;                                            // [8][16][64]
    double *s_x = s_out + SP_THREADS * 16;                            // [n + 1][BN], last row ones
    unsigned short *s_vd = (unsigned short *)(s_x + (n + 1) * SP_BN); // [2][S][BN][SP_LDK]
    uint4 *s_enc = (uint4 *)(s_vd + 2 * S * SP_BN * SP_LDK);         // [2][SP_KS]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * SP_BM;
    const int64_t n0 = (int64_t)blockIdx.x * SP_BN;
    const int64_t RB = ceil_div(P, 32);
    const int64_t KC = Kp >> 4;
    for (int idx = tid; idx < (n + 1) * SP_BN; idx += SP_THREADS) {
        const int i = idx / SP_BN, c = idx % SP_BN;
        const int64_t pt = n0 + c;
        s_x[idx] = i == n ? 1.0 : (pt < N ? X[pt * n + i] : 0.0);
    }
    double out[16];                                 // tile 0 sums; tile 1 sums in s_out
    double *my_out = s_out + w * 16 * 64 + lane;    // element v at my_out[64 v]
    f16v acc[SP_GROUPS][2];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        out[v] = 0.0;
        my_out[64 * v] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < SP_GROUPS; ++g)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[g][ct][v] = 0.0f;

    // C digits of this wave: plane s, row block r0 / 32 + w.  One buffer per
    // plane over the workgroup's row blocks that exist (waves past P read
    // zeros; a load past Kp reads the next row block or zeros, never used);
    // byte offsets stay below 2^31 (host check on Kp).
    const int64_t rb0 = r0 >> 5;
    const int nrb = (int)(RB - rb0 < SP_BM / 32 ? RB - rb0 : SP_BM / 32);
    const int aoff = ((w * (int)KC) * 64 + lane) * 16;
    u32x4 A[2][S];
    auto load_a = [&](int64_t kk) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(Cs + ((s * RB + rb0) * KC << 9)), (short)0, nrb * (int)KC * 1024, 0x00020000);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                A[j][s] = __builtin_amdgcn_raw_buffer_load_b128(rs, aoff + (int)((kk >> 4) + j) * 1024, 0, 0);
        }
    };
    // factor lists of step kk (lanes tid < SP_KS; zero past K) and the scale
    // exponent of this thread's point for the K-block of step kk
    uint4 ereg = make_uint4(0, 0, 0, 0);
    auto load_enc = [&](int64_t kk) {
        if (tid < SP_KS) {
            const __amdgpu_buffer_rsrc_t re = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(enc + kk), (short)0, (int)((K - kk) * 16 > 0 ? (K - kk) * 16 : 0), 0x00020000);
            const u32x4 e = __builtin_amdgcn_raw_buffer_load_b128(re, tid * 16, 0, 0);
            ereg = make_uint4(e[0], e[1], e[2], e[3]);
        }
    };
    const int vc = tid % SP_BN;
    const int vkq = (tid / SP_BN) * SP_VK;
    const int64_t vpt = n0 + vc;
    auto load_sig = [&](int64_t kk) -> int {   // points past N, steps past Kp read zero; never used
        const int nrec = kk < Kp ? (int)((N - n0 < SP_BN ? N - n0 : SP_BN) * 4) : 0;
        const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(sig_v + (kk < Kp ? (kk / DN_KB) * N + n0 : 0)), (short)0, nrec, 0x00020000);
        return (int)__builtin_amdgcn_raw_buffer_load_b32(rg, vc * 4, 0, 0);
    };
    // V digits of step kk (this thread: point vc, k = kk + vkq .. + 3) into
    // buffer vb.  general = false: one factor word (exact for degree <= 4).
    auto gen_v = [&](int64_t kk, int sig, int vb, bool general) {
        const bool live = vpt < N && sig > -1100;
        const uint4 *le = s_enc + vb * SP_KS;
        float scale[S];
#pragma unroll
        for (int t = 0; t < S; ++t) scale[t] = live ? ldexpf(1.0f, sig - 8 * (t + 1)) : 0.0f;
        uint32_t dig[S][SP_VK / 2];
#pragma unroll
        for (int q = 0; q < SP_VK; ++q) {
            const int64_t k = kk + vkq + q;
            double y;
            if (general) {
                y = 0.0;
                if (live && k < K) y = ldexp(factor_value(le[vkq + q], basis + k * n, n, s_x + vc, SP_BN), -sig);
            } else {
                // masked by bits, not by a branch or a product, so the block
                // stays straight-line and a masked value is exactly 0
                const double v = factor_chunk(1.0, le[vkq + q].x, s_x + vc, SP_BN);
                const uint64_t keep = (live && k < K) ? ~0ull : 0ull;
                y = ldexp(__builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & keep), -sig);
            }
            put_digits<S>(y, scale, q, dig);
        }
#pragma unroll
        for (int d = 0; d < S; ++d)
            *(uint2 *)(s_vd + ((vb * S + d) * SP_BN + vc) * SP_LDK + vkq) = make_uint2(dig[d][0], dig[d][1]);
    };
    auto redo_high_degree = [&](int64_t kk, int sig, int vb) {
        const uint4 *le = s_enc + vb * SP_KS;
        bool high = false;
#pragma unroll
        for (int q = 0; q < SP_VK; ++q) high |= le[vkq + q].w > 4u && kk + vkq + q < K;
        if (high) gen_v(kk, sig, vb, true);
    };
    auto mfma_step = [&](int vb) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int t = 0; t < S; ++t) {
                s8v b[2];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
                    b[ct] = *(const s8v *)(s_vd + ((vb * S + t) * SP_BN + ct * 32 + (lane & 31)) * SP_LDK + 16 * j +
                                           8 * (lane >> 5));
#pragma unroll
                for (int s = 0; s < S - t; ++s) {
                    const int g = (s + t) < SP_GROUPS - 1 ? (s + t) : SP_GROUPS - 1;
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[g][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf8v, A[j][s]), __builtin_bit_cast(bf8v, b[ct]), acc[g][ct], 0, 0, 0);
                }
            }
        }
    };
    auto fold = [&]() {   // close a K-block: FP32 groups into the FP64 sums
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                double t = 0.0;
#pragma unroll
                for (int g = SP_GROUPS - 1; g >= 0; --g) {
                    t += (double)acc[g][ct][v];
                    acc[g][ct][v] = 0.0f;
                }
                if (ct == 0) out[v] += t;
                else my_out[64 * v] += t;
            }
    };

    // prologue: factor lists of steps 0 and 1 staged, V tile of step 0 formed
    load_a(0);
    load_enc(0);
    int sg = load_sig(0);
    __syncthreads();
    if (tid < SP_KS) s_enc[tid] = ereg;
    load_enc(SP_KS);
    __syncthreads();
    gen_v(0, sg, 0, false);
    redo_high_degree(0, sg, 0);
    if (tid < SP_KS) s_enc[SP_KS + tid] = ereg;
    load_enc(2 * SP_KS);
    sg = load_sig(SP_KS);   // during step i: the scale of step i + 1
    __syncthreads();
    const int64_t nsteps = Kp / SP_KS;
    for (int64_t i = 0; i < nsteps; ++i) {
        const int64_t k1 = (i + 1) * SP_KS;
        const int vb = (int)(i & 1);
        mfma_step(vb);
        load_a(k1);
        gen_v(k1, sg, vb ^ 1, false);
        redo_high_degree(k1, sg, vb ^ 1);
        if ((k1 % DN_KB) == 0 || i + 1 == nsteps) fold();
        // factor lists of step i + 2 into the buffer step i's lists leave
        // (those of step i + 3 in flight), and the scale of step i + 2
        if (tid < SP_KS) s_enc[vb * SP_KS + tid] = ereg;
        load_enc(k1 + 2 * SP_KS);
        sg = load_sig(k1 + SP_KS);
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t r = r0 + w * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int64_t c = n0 + ct * 32 + (lane & 31);
            if (r < P && c < N) Y[(r * N + c) * ys] = ct == 0 ? out[v] : my_out[64 * v];
        }
}

// ------------------------------------------------- split reverse mode: dC
//
// dC = gY V^T on the same splitting with the operands' roles moved: the
// contraction runs over points in blocks of DN_KB.  gY [P x N] is cut into
// digit planes by k_split_c (one scale per row and point block); V^T gets one
// scale per monomial and point block, written by k_split_wscale, and its
// digits are formed per step in LDS.  The error bound is the forward's with
// sum_pt |gY v| in place of sum_k |C v|.

// Scales of V^T: sig_w[pb * K + k] = exponent above max |v_k(x_pt)| over the
// points pt of block pb.  One block per (point block, 256 monomials), one
// monomial per thread; the block's points sit point-major in LDS ([DN_KB][n +
// 1], last entry of each point one), so a wave reads one point's
// coordinates, each lane the variables its monomial names.
__global__ void __launch_bounds__(256) k_split_wscale(int n, int64_t K, const uint8_t *basis, const uint4 *enc,
                                                      int64_t N, const double *X, int32_t *sig_w)
{
    extern __shared__ double s_pt[];   // [DN_KB][n + 1]
    const int64_t ktiles = ceil_div(K, 256);
    const int64_t pb = blockIdx.x / ktiles;
    const int64_t k = (blockIdx.x % ktiles) * 256 + threadIdx.x;
    const int64_t p0 = pb * DN_KB;
    const int np1 = n + 1;
    for (int idx = threadIdx.x; idx < DN_KB * np1; idx += 256) {
        const int l = idx / np1, i = idx % np1;
        s_pt[idx] = i == n ? 1.0 : (p0 + l < N ? X[(p0 + l) * n + i] : 0.0);
    }
    __syncthreads();
    if (k >= K) return;
    const uint4 e = enc[k];
    const int npts = (int)(N - p0 < DN_KB ? N - p0 : DN_KB);
    double amax = 0.0;
    for (int l = 0; l < npts; ++l) amax = fmax(amax, fabs(factor_value(e, basis + k * n, n, s_pt + l * np1, 1)));
    sig_w[pb * K + k] = scale_exp(amax);
}

// coordinates per thread per step: XR = 2 for n <= 32, 4 for n <= 64
constexpr int SW_XR_MAX = 4;

__host__ __device__ constexpr size_t split_dc_lds_bytes(int n, int S)
{
    return (size_t)SP_THREADS * 16 * 8 + (size_t)2 * SP_KS * (n + 1) * 8 + (size_t)2 * S * SP_BN * SP_LDK * 2;
}

// grid: x = monomial tiles of SP_BN, y = row tiles of SP_BM.  The tile shape,
// accumulator groups, K-block folds and double buffering are those of
// k_dense_split with points as the contraction: wave w owns rows r0 + 32 w
// .. + 31 and the workgroup's SP_BN monomials; its gY digits come from the
// MFMA-ordered planes (Np = N padded to SP_KS) into registers.  Each thread
// owns one monomial (its factor list stays in registers) and forms its
// digits at 4 of a step's SP_KS points; the step's coordinates, SP_KS * n
// consecutive doubles of X, are loaded into registers a step ahead and
// stored point-major into LDS.  Dynamic LDS: FP64 sums [8 waves][16][64
// lanes], points [2][SP_KS][n + 1] doubles, digits [2][S][BN][SP_LDK] bf16.
template <int S, int XR>
__global__ void __launch_bounds__(SP_THREADS) k_dense_bwd_dc_split(int n, int64_t K, const uint8_t *basis,
                                                                   const uint4 *enc, int64_t P,
                                                                   const unsigned short *Gs, int64_t N, int64_t Np,
                                                                   const double *X, const int32_t *sig_w, double *dC)
{
    static_assert(SP_VK == 4, "V digits are stored as 2 words per plane");
    extern __shared__ double s_dyn[];
    const int np1 = n + 1;
    double *s_out = s_dyn;                                                   // [8][16][64]
    double *s_xp = s_out + SP_THREADS * 16;                                  // [2][SP_KS][n + 1]
    unsigned short *s_vd = (unsigned short *)(s_xp + 2 * SP_KS * np1);      // [2][S][BN][SP_LDK]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * SP_BM;
    const int64_t k0 = (int64_t)blockIdx.x * SP_BN;
    const int64_t RB = ceil_div(P, 32);
    const int64_t KC = Np >> 4;
    for (int idx = tid; idx < 2 * SP_KS; idx += SP_THREADS) s_xp[idx * np1 + n] = 1.0;
    double out[16];
    double *my_out = s_out + w * 16 * 64 + lane;
    f16v acc[SP_GROUPS][2];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        out[v] = 0.0;
        my_out[64 * v] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < SP_GROUPS; ++g)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[g][ct][v] = 0.0f;

    // gY digits of this wave (as the C digits of k_dense_split; the host
    // keeps a workgroup's rows of one plane below 2^31 bytes)
    const int64_t rb0 = r0 >> 5;
    const int nrb = (int)(RB - rb0 < SP_BM / 32 ? RB - rb0 : SP_BM / 32);
    const int aoff = ((w * (int)KC) * 64 + lane) * 16;
    u32x4 A[2][S];
    auto load_a = [&](int64_t kk) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(Gs + ((s * RB + rb0) * KC << 9)), (short)0, nrb * (int)KC * 1024, 0x00020000);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                A[j][s] = __builtin_amdgcn_raw_buffer_load_b128(rs, aoff + (int)((kk >> 4) + j) * 1024, 0, 0);
        }
    };
    // this thread's monomial and its slots of a step's points
    const int vc = tid % SP_BN;
    const int vkq = (tid / SP_BN) * SP_VK;
    const int64_t kcol = k0 + vc;
    const uint4 my_enc = kcol < K ? enc[kcol] : make_uint4(0, 0, 0, 0);
    const bool high = my_enc.w > 4u;
    const uint8_t *my_row = basis + (kcol < K ? kcol : 0) * n;
    // coordinates of step kk: element e = l * n + i of the step's block of
    // X (point kk + l, variable i), elements tid + r * SP_THREADS; past N zero
    double xr[XR];
    int xo[XR];
#pragma unroll
    for (int r = 0; r < XR; ++r) {
        const int e = tid + r * SP_THREADS;
        xo[r] = e < SP_KS * n ? (e / n) * np1 + e % n : -1;
    }
    auto load_x = [&](int64_t kk) {
        const int64_t left = kk < N ? (N - kk) * n * 8 : 0;
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(X + (kk < N ? kk * n : 0)), (short)0, (int)(left < SP_KS * n * 8 ? left : SP_KS * n * 8),
            0x00020000);
#pragma unroll
        for (int r = 0; r < XR; ++r)
            xr[r] = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rx, (tid + r * SP_THREADS) * 8, 0, 0));
    };
    auto store_x = [&](int buf) {
#pragma unroll
        for (int r = 0; r < XR; ++r)
            if (xo[r] >= 0) s_xp[buf * SP_KS * np1 + xo[r]] = xr[r];
    };
    auto load_sig = [&](int64_t kk) -> int {   // monomials past K, steps past Np read zero; never used
        const int nrec = kk < Np ? (int)((K - k0 < SP_BN ? K - k0 : SP_BN) * 4) : 0;
        const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(sig_w + (kk < Np ? (kk / DN_KB) * K + k0 : 0)), (short)0, nrec, 0x00020000);
        return (int)__builtin_amdgcn_raw_buffer_load_b32(rg, vc * 4, 0, 0);
    };
    // digits of v_kcol at points kk + vkq .. + 3 (points of buffer vb) into
    // digit buffer vb.  general = false: one factor word (degree <= 4).
    auto gen_v = [&](int64_t kk, int sig, int vb, bool general) {
        const bool live = kcol < K && sig > -1100;
        const double *xb = s_xp + vb * SP_KS * np1;
        float scale[S];
#pragma unroll
        for (int t = 0; t < S; ++t) scale[t] = live ? ldexpf(1.0f, sig - 8 * (t + 1)) : 0.0f;
        uint32_t dig[S][SP_VK / 2];
#pragma unroll
        for (int q = 0; q < SP_VK; ++q) {
            const int64_t pt = kk + vkq + q;
            const double *xq = xb + (vkq + q) * np1;
            double y;
            if (general) {
                y = 0.0;
                if (live && pt < N) y = ldexp(factor_value(my_enc, my_row, n, xq, 1), -sig);
            } else {
                const double v = factor_chunk(1.0, my_enc.x, xq, 1);
                const uint64_t keep = (live && pt < N) ? ~0ull : 0ull;
                y = ldexp(__builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & keep), -sig);
            }
            put_digits<S>(y, scale, q, dig);
        }
#pragma unroll
        for (int d = 0; d < S; ++d)
            *(uint2 *)(s_vd + ((vb * S + d) * SP_BN + vc) * SP_LDK + vkq) = make_uint2(dig[d][0], dig[d][1]);
    };
    auto mfma_step = [&](int vb) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int t = 0; t < S; ++t) {
                s8v b[2];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
                    b[ct] = *(const s8v *)(s_vd + ((vb * S + t) * SP_BN + ct * 32 + (lane & 31)) * SP_LDK + 16 * j +
                                           8 * (lane >> 5));
#pragma unroll
                for (int s = 0; s < S - t; ++s) {
                    const int g = (s + t) < SP_GROUPS - 1 ? (s + t) : SP_GROUPS - 1;
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[g][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf8v, A[j][s]), __builtin_bit_cast(bf8v, b[ct]), acc[g][ct], 0, 0, 0);
                }
            }
        }
    };
    auto fold = [&]() {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                double t = 0.0;
#pragma unroll
                for (int g = SP_GROUPS - 1; g >= 0; --g) {
                    t += (double)acc[g][ct][v];
                    acc[g][ct][v] = 0.0f;
                }
                if (ct == 0) out[v] += t;
                else my_out[64 * v] += t;
            }
    };

    // prologue: points of steps 0 and 1 staged, digits of step 0 formed
    load_a(0);
    load_x(0);
    int sg = load_sig(0);
    __syncthreads();
    store_x(0);
    load_x(SP_KS);
    __syncthreads();
    gen_v(0, sg, 0, false);
    if (high) gen_v(0, sg, 0, true);
    store_x(1);
    load_x(2 * SP_KS);
    sg = load_sig(SP_KS);   // during step i: the scale of step i + 1
    __syncthreads();
    const int64_t nsteps = Np / SP_KS;
    for (int64_t i = 0; i < nsteps; ++i) {
        const int64_t k1 = (i + 1) * SP_KS;
        const int vb = (int)(i & 1);
        mfma_step(vb);
        load_a(k1);
        gen_v(k1, sg, vb ^ 1, false);
        if (high) gen_v(k1, sg, vb ^ 1, true);
        if ((k1 % DN_KB) == 0 || i + 1 == nsteps) fold();
        // points of step i + 2 into the buffer step i's points leave (those
        // of step i + 3 in flight), and the scale of step i + 2
        store_x(vb);
        load_x(k1 + 2 * SP_KS);
        sg = load_sig(k1 + SP_KS);
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t r = r0 + w * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int64_t c = k0 + ct * 32 + (lane & 31);
            if (r < P && c < K) dC[r * K + c] = ct == 0 ? out[v] : my_out[64 * v];
        }
}

// ------------------------------------------------- split reverse mode: dX
//
// dX[pt][j] = sum_k W[k][pt] d v_k / d x_j (x_pt), W = C^T gY.  The split
// form computes W for a chunk of points as a plain product of two given
// matrices on the splitting above, contraction over the polynomials in
// blocks of DN_KB: C^T and gY^T are cut into digit planes (rows monomials,
// resp. points; one scale per row and polynomial block) by k_split_ct; W
// [K x chunk] is stored in FP64; a second pass contracts it with the
// monomials' derivatives, K split over blocks whose partial sums are added
// in a fixed order.

// Digit planes (split_c_index order) of the transpose of a row-major matrix:
// row r, column kk of the operand is M[kk * ld + r], r < R, kk < Kc; rows up
// to ceil(R / 32) * 32 and columns up to Kp (multiple of SP_KS) are padded
// with zero digits.  One block per (32 rows, DN_KB columns): the tile is
// read along r (coalesced) into LDS, each thread then owns one column.
__global__ void __launch_bounds__(DN_KB) k_split_ct(const double *M, int64_t ld, int64_t R, int64_t Kc, int64_t Kp,
                                                    int S, unsigned short *Ms)
{
    __shared__ double s_t[DN_KB][33];
    __shared__ double s_m[4][32];
    const int64_t nkb = ceil_div(Kp, DN_KB);
    const int64_t RB = ceil_div(R, 32);
    const int64_t rb = blockIdx.x / nkb, kb = blockIdx.x % nkb;
    const int64_t r0 = rb * 32, k0 = kb * DN_KB;
    const int t = threadIdx.x;
    for (int idx = t; idx < DN_KB * 32; idx += DN_KB) {
        const int kk = idx >> 5, r = idx & 31;
        s_t[kk][r] = (r0 + r < R && k0 + kk < Kc) ? M[(k0 + kk) * ld + r0 + r] : 0.0;
    }
    __syncthreads();
    {
        const int r = t & 31, g = t >> 5;
        double a = 0.0;
        for (int q = 0; q < 32; ++q) a = fmax(a, fabs(s_t[g * 32 + q][r]));
        s_m[g][r] = a;
    }
    __syncthreads();
    const int64_t k = k0 + t;
    if (k >= Kp) return;
    for (int r = 0; r < 32; ++r) {
        const double amax = fmax(fmax(s_m[0][r], s_m[1][r]), fmax(s_m[2][r], s_m[3][r]));
        const int sig = scale_exp(amax);
        double y = amax > 0.0 ? ldexp(s_t[t][r], -sig) : 0.0;
        for (int d = 1; d <= S; ++d) {
            y = y * 256.0;
            const double m = rint(y);
            y = y - m;
            Ms[split_c_index(d - 1, r0 + r, k, RB, Kp)] = bf16_bits_exact(ldexpf((float)m, sig - 8 * d));
        }
    }
}

constexpr int SG_REC = 64 * 16;   // bytes of one operand record (64 lanes x 8 BF16)

__host__ __device__ constexpr size_t split_gemm_lds_bytes(int S)
{
    return (size_t)SP_THREADS * 16 * 8 + (size_t)2 * 4 * S * SG_REC;
}

// out[r * ldo + c] = sum_kk A[r][kk] B[c][kk] for r < R, c < Cn, with A and
// B given as digit planes (split_c_index order, RBa resp. RBb row blocks,
// Kp columns); columns are those of B's row blocks cb0 .. of this launch.
// grid: x = column tiles of SP_BN, y = row tiles of SP_BM.  The tile shape,
// accumulator groups and K-block folds are k_dense_split's; wave w's A
// digits come straight into registers, and the workgroup's B records (2
// column blocks x S planes x 2 chunks of 16 per step) are staged in LDS,
// loaded into registers a step ahead.  Dynamic LDS: FP64 sums [8][16][64],
// B records [2][2 * S * 2][64 lanes][16 B].
template <int S>
__global__ void __launch_bounds__(SP_THREADS) k_split_gemm(int64_t R, int64_t RBa, const unsigned short *As,
                                                           int64_t Cn, int64_t RBb, int64_t cb0,
                                                           const unsigned short *Bs, int64_t Kp, double *out,
                                                           int64_t ldo)
{
    constexpr int NREC = 2 * S * 2;                              // records per step
    constexpr int BR = (NREC * 64 + SP_THREADS - 1) / SP_THREADS;  // record loads per thread
    extern __shared__ double s_dyn[];
    double *s_out = s_dyn;                                    // [8][16][64]
    u32x4 *s_b = (u32x4 *)(s_out + SP_THREADS * 16);          // [2][NREC][64]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * SP_BM;
    const int64_t cblk0 = cb0 + (int64_t)blockIdx.x * 2;      // first of the tile's two column blocks
    const int64_t KC = Kp >> 4;
    double out_r[16];
    double *my_out = s_out + w * 16 * 64 + lane;
    f16v acc[SP_GROUPS][2];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        out_r[v] = 0.0;
        my_out[64 * v] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < SP_GROUPS; ++g)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[g][ct][v] = 0.0f;
    const int64_t rb0 = r0 >> 5;
    const int nrb = (int)(RBa - rb0 < SP_BM / 32 ? RBa - rb0 : SP_BM / 32);
    const int aoff = ((w * (int)KC) * 64 + lane) * 16;
    u32x4 A[2][S];
    auto load_a = [&](int64_t kk) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(As + ((s * RBa + rb0) * KC << 9)), (short)0, nrb * (int)KC * 1024, 0x00020000);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                A[j][s] = __builtin_amdgcn_raw_buffer_load_b128(rs, aoff + (int)((kk >> 4) + j) * 1024, 0, 0);
        }
    };
    // record q = (ct * S + t) * 2 + j of step kk: plane t, column block
    // cblk0 + ct, chunk kk / 16 + j; blocks past RBb and steps past Kp read zero
    u32x4 breg[BR];
    auto load_b = [&](int64_t kk) {
#pragma unroll
        for (int m = 0; m < BR; ++m) {
            const int q = (tid >> 6) + m * (SP_THREADS / 64);
            breg[m] = (u32x4){0u, 0u, 0u, 0u};
            if (q < NREC) {
                const int j = q & 1, t = (q >> 1) % S, ct = (q >> 1) / S;
                const int64_t cblk = cblk0 + ct;
                const int nrec = (cblk < RBb && kk < Kp) ? (int)(KC * 1024) : 0;
                const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(Bs + ((t * RBb + (cblk < RBb ? cblk : 0)) * KC << 9)), (short)0, nrec, 0x00020000);
                breg[m] = __builtin_amdgcn_raw_buffer_load_b128(rb, (int)((kk >> 4) + j) * 1024 + lane * 16, 0, 0);
            }
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int m = 0; m < BR; ++m) {
            const int q = (tid >> 6) + m * (SP_THREADS / 64);
            if (q < NREC) s_b[(buf * NREC + q) * 64 + lane] = breg[m];
        }
    };
    auto mfma_step = [&](int vb) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int t = 0; t < S; ++t) {
                u32x4 b[2];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) b[ct] = s_b[(vb * NREC + (ct * S + t) * 2 + j) * 64 + lane];
#pragma unroll
                for (int s = 0; s < S - t; ++s) {
                    const int g = (s + t) < SP_GROUPS - 1 ? (s + t) : SP_GROUPS - 1;
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[g][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf8v, A[j][s]), __builtin_bit_cast(bf8v, b[ct]), acc[g][ct], 0, 0, 0);
                }
            }
        }
    };
    auto fold = [&]() {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                double t = 0.0;
#pragma unroll
                for (int g = SP_GROUPS - 1; g >= 0; --g) {
                    t += (double)acc[g][ct][v];
                    acc[g][ct][v] = 0.0f;
                }
                if (ct == 0) out_r[v] += t;
                else my_out[64 * v] += t;
            }
    };
    load_a(0);
    load_b(0);
    __syncthreads();
    store_b(0);
    load_b(SP_KS);
    __syncthreads();
    const int64_t nsteps = Kp / SP_KS;
    for (int64_t i = 0; i < nsteps; ++i) {
        const int64_t k1 = (i + 1) * SP_KS;
        const int vb = (int)(i & 1);
        mfma_step(vb);
        load_a(k1);
        store_b(vb ^ 1);          // B of step i + 1 (its buffer held step i - 1's)
        load_b(k1 + SP_KS);
        if ((k1 % DN_KB) == 0 || i + 1 == nsteps) fold();
        __syncthreads();
    }
    const int64_t c0 = (cblk0 - cb0) * 32;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t r = r0 + w * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int64_t c = c0 + ct * 32 + (lane & 31);
            if (r < R && c < Cn) out[r * ldo + c] = ct == 0 ? out_r[v] : my_out[64 * v];
        }
}

constexpr int DW_WAVES = 4, DW_KSPLIT = 16;

// Partial dX of a chunk of points from W [K x ldw] (FP64): block (point
// tile of 64, K range q of DW_KSPLIT), wave w the w-th quarter of that range;
// lane = point.  Each wave adds W[k][pt] d v_k / d x_j into its accumulator
// block [n][64] in LDS in the order of k, then the four blocks are added in
// wave order into part[q][pt][j].  Dynamic LDS: points [n + 1][64] (last row
// ones), accumulators [DW_WAVES][n][64].
__global__ void __launch_bounds__(DW_WAVES * 64) k_dx_from_w(int n, int64_t K, const uint8_t *basis,
                                                             const uint64_t *senc, const double *W, int64_t ldw,
                                                             int64_t Nc, const double *X, double *part)
{
    extern __shared__ double s_dyn[];
    double *s_x = s_dyn;                              // [n + 1][64]
    double *s_acc = s_dyn + (size_t)(n + 1) * 64;     // [DW_WAVES][n][64]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int q = blockIdx.y;
    for (int idx = tid; idx < (n + 1) * 64; idx += DW_WAVES * 64) {
        const int i = idx / 64, c = idx % 64;
        s_x[idx] = i == n ? 1.0 : (p0 + c < Nc ? X[(p0 + c) * n + i] : 0.0);
    }
    for (int idx = tid; idx < DW_WAVES * n * 64; idx += DW_WAVES * 64) s_acc[idx] = 0.0;
    __syncthreads();
    const int64_t per = ceil_div(K, (int64_t)DW_KSPLIT * DW_WAVES);
    const int64_t kb = ((int64_t)q * DW_WAVES + w) * per;
    const int64_t ke = kb + per < K ? kb + per : K;
    const int64_t pt = p0 + lane;
    double *my_acc = s_acc + (size_t)w * n * 64 + lane;
    if (pt < Nc)
        for (int64_t k = kb; k < ke; ++k) {
            const double wv = W[k * ldw + pt];
            add_monomial_grad(senc[2 * k], senc[2 * k + 1], basis + k * n, n, s_x + lane, 64, wv, my_acc);
        }
    __syncthreads();
    for (int idx = tid; idx < 64 * n; idx += DW_WAVES * 64) {
        const int pl = idx / n, j = idx % n;
        if (p0 + pl >= Nc) continue;
        double a = 0.0;
#pragma unroll
        for (int ww = 0; ww < DW_WAVES; ++ww) a += s_acc[((size_t)ww * n + j) * 64 + pl];
        part[((size_t)q * Nc + p0 + pl) * n + j] = a;
    }
}

// dX rows of a chunk: the DW_KSPLIT partial sums added in order
__global__ void k_dx_reduce(const double *part, int64_t Nc, int n, double *dX)
{
    const int64_t m = Nc * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int q = 0; q < DW_KSPLIT; ++q) a += part[q * m + i];
        dX[i] = a;
    }
}

// ---------------------------------------------------------------- host side

namespace {

struct DensePlan {
    size_t enc, cs, sigv, total;
};

DensePlan plan_dense(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t S)
{
    size_t off = kWsHeadBytes;
    auto take = [&](size_t b) {
        const size_t o = align_up(off, 256);
        off = o + b;
        return o;
    };
    DensePlan d;
    d.enc = take(16 * (size_t)K);
    d.cs = 0;
    d.sigv = 0;
    if (prec == POLY_SPLIT_BF16) {
        const int64_t Kp = align_up((size_t)K, 32);
        d.cs = take((size_t)S * ceil_div(P, 32) * 32 * Kp * 2);
        d.sigv = take((size_t)ceil_div(Kp, DN_KB) * N * 4);
    }
    d.total = align_up(off, 256);
    return d;
}

template <int S>
void launch_split(int n, int64_t K, int64_t Kp, const uint8_t *basis, const uint4 *enc, int64_t P,
                  const unsigned short *Cs, int64_t N, const double *X, const int32_t *sig_v, double *Y, int64_t ys,
                  hipStream_t s)
{
    const size_t lds = split_lds_bytes(n, S);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_dense_split<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    const dim3 grid((unsigned)ceil_div(N, SP_BN), (unsigned)ceil_div(P, SP_BM));
    TimedLaunch tl(POLY_TIMING_DENSE, s);
    hipLaunchKernelGGL((k_dense_split<S>), grid, dim3(SP_THREADS), lds, s, n, K, Kp, basis, enc, P, Cs, N, X, sig_v,
                       Y, ys);
    tl.done(s);
}

}  // namespace

poly_status dense_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t S, size_t *ws_bytes)
{
    if (!ws_bytes || n < 1 || n > 255 || K < 0 || P < 0 || N < 0) return POLY_ERR_ARG;
    if (prec != POLY_FP64 && prec != POLY_SPLIT_BF16) return POLY_ERR_ARG;
    if (prec == POLY_SPLIT_BF16 && (S < 3 || S > 5)) return POLY_ERR_ARG;
    *ws_bytes = plan_dense(n, K, P, N, prec, S).total;
    return POLY_OK;
}

poly_status dense_run(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P, const double *C,
                      int64_t N, const double *X, double *Y, poly_prec prec, int32_t S, void *ws, size_t ws_bytes,
                      hipStream_t s, int64_t ys)
{
    size_t need = 0;
    poly_status st = dense_workspace(n, K, P, N, prec, S, &need);
    if (st != POLY_OK) return st;
    if (max_exp < 0 || max_exp > 255) return POLY_ERR_ARG;
    if ((K > 0 && (!basis || (P > 0 && !C))) || (N > 0 && !X) || (P > 0 && N > 0 && !Y)) return POLY_ERR_ARG;
    if (!ws || ws_bytes < need) return POLY_ERR_WORKSPACE;
    if (prec == POLY_FP64 && (size_t)(n + 1) * D64_BN * 8 > 96 * 1024) return POLY_ERR_UNSUPPORTED;
    if (prec == POLY_SPLIT_BF16 && split_lds_bytes(n, S) > 160 * 1024) return POLY_ERR_UNSUPPORTED;
    // both kernels address one block's rows of C (up to 128 x K doubles, or
    // 256 x Kp BF16 digits of one plane) with 32-bit byte offsets
    const int bm = prec == POLY_FP64 && tunables().dense_f64_rows == 128 ? 128 : 64;
    if ((int64_t)align_up((size_t)K, 32) * 8 * bm + 256 > INT32_MAX) return POLY_ERR_UNSUPPORTED;
    const DensePlan d = plan_dense(n, K, P, N, prec, S);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)ws, 0ull, (int64_t)1);
    if (P == 0 || N == 0) return hipGetLastError() == hipSuccess ? POLY_OK : POLY_ERR_HIP;
    uint4 *enc = (uint4 *)((char *)ws + d.enc);
    if (K > 0)
        hipLaunchKernelGGL(k_encode_factors, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, basis, K, n,
                           (uint32_t *)enc, (const int64_t *)nullptr, (uint32_t *)nullptr);
    if (prec == POLY_FP64) {
        static bool attr = false;
        if (!attr) {
            // the points tile is at most 96 KB (checked above); with the static
            // tiles of the 128-row form that is within the 160 KB of a CU
            (void)hipFuncSetAttribute((const void *)k_dense_f64<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      96 * 1024);
            (void)hipFuncSetAttribute((const void *)k_dense_f64<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      96 * 1024);
            attr = true;
        }
        const dim3 grid((unsigned)ceil_div(N, D64_BN), (unsigned)ceil_div(P, bm));
        TimedLaunch tl(POLY_TIMING_DENSE, s);
        if (bm == 128)
            hipLaunchKernelGGL(k_dense_f64<128>, grid, dim3(D64_THREADS), (size_t)(n + 1) * D64_BN * 8, s, n, K,
                               basis, (const uint4 *)enc, P, C, N, X, Y, ys);
        else
            hipLaunchKernelGGL(k_dense_f64<64>, grid, dim3(D64_THREADS), (size_t)(n + 1) * D64_BN * 8, s, n, K,
                               basis, (const uint4 *)enc, P, C, N, X, Y, ys);
        tl.done(s);
    } else {
        unsigned short *Cs = (unsigned short *)((char *)ws + d.cs);
        int32_t *sig_v = (int32_t *)((char *)ws + d.sigv);
        const int64_t Kp = align_up((size_t)K, 32);
        const int64_t nkb = ceil_div(Kp, DN_KB);
        if (K > 0) {
            hipLaunchKernelGGL(k_split_c, dim3((unsigned)(ceil_div(P, 32) * 32 * nkb)), dim3(DN_KB), 0, s, C, P, K,
                               Kp, S, Cs);
            hipLaunchKernelGGL(k_split_vscale, dim3((unsigned)(nkb * ceil_div(N, 64))), dim3(256),
                               (size_t)(n + 1) * 64 * 8, s, n, K, basis, (const uint4 *)enc, N, X, sig_v);
        }
        switch (S) {
        case 3: launch_split<3>(n, K, Kp, basis, enc, P, Cs, N, X, sig_v, Y, ys, s); break;
        case 4: launch_split<4>(n, K, Kp, basis, enc, P, Cs, N, X, sig_v, Y, ys, s); break;
        default: launch_split<5>(n, K, Kp, basis, enc, P, Cs, N, X, sig_v, Y, ys, s); break;
        }
    }
    return hipGetLastError() == hipSuccess ? POLY_OK : POLY_ERR_HIP;
}

// ------------------------------------------------- reverse mode: host side

// dynamic LDS of the dX kernel: points [(n + 1)][128], four accumulator blocks [n][64]
inline size_t dense_bwd_dx_lds(int n) { return ((size_t)(n + 1) * DB_BN + 4 * (size_t)n * kWave) * 8; }
constexpr size_t DB_DX_LDS_MAX = 130 * 1024;   // beside ~27 KB of static LDS

namespace {

constexpr int64_t DX_CHUNK = 4096;   // points per W chunk of the split dX

struct DenseBwdPlan {
    size_t fenc, senc, gs, sigw, ct, gyt, w, part, total;
    int64_t Np, Pp, Nc;
};

// workspace: status word, factor lists and support encodings of the basis;
// split: for dC the gY digit planes [S][ceil(P / 32) * 32][Np] and the scales
// of V^T [ceil(N / DN_KB)][K]; for dX the digit planes of C^T [S][ceil(K /
// 32) * 32][Pp] and of gY^T [S][ceil(N / 32) * 32][Pp], one W chunk [K][Nc]
// and the partial sums [DW_KSPLIT][Nc][n]
DenseBwdPlan plan_dense_bwd(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t S)
{
    size_t off = kWsHeadBytes;
    auto take = [&](size_t b) {
        const size_t o = align_up(off, 256);
        off = o + b;
        return o;
    };
    DenseBwdPlan d;
    d.fenc = take(16 * (size_t)K);
    d.senc = take(16 * (size_t)K);
    d.gs = d.sigw = d.ct = d.gyt = d.w = d.part = 0;
    d.Np = (int64_t)align_up((size_t)N, SP_KS);
    d.Pp = (int64_t)align_up((size_t)P, SP_KS);
    d.Nc = std::min<int64_t>((int64_t)align_up((size_t)N, 64), DX_CHUNK);
    if (prec == POLY_SPLIT_BF16) {
        d.gs = take((size_t)S * ceil_div(P, 32) * 32 * d.Np * 2);
        d.sigw = take((size_t)ceil_div(N, DN_KB) * K * 4);
        d.ct = take((size_t)S * ceil_div(K, 32) * 32 * d.Pp * 2);
        d.gyt = take((size_t)S * ceil_div(N, 32) * 32 * d.Pp * 2);
        d.w = take((size_t)K * d.Nc * 8);
        d.part = take((size_t)DW_KSPLIT * d.Nc * n * 8);
    }
    d.total = align_up(off, 256);
    return d;
}

template <int S, int XR>
void launch_bwd_dc_split_xr(int n, int64_t K, const uint8_t *basis, const uint4 *enc, int64_t P,
                         const unsigned short *Gs, int64_t N, int64_t Np, const double *X, const int32_t *sig_w,
                         double *dC, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_dense_bwd_dc_split<S, XR>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    const dim3 grid((unsigned)ceil_div(K, SP_BN), (unsigned)ceil_div(P, SP_BM));
    TimedLaunch tl(POLY_TIMING_DENSE, s);
    hipLaunchKernelGGL((k_dense_bwd_dc_split<S, XR>), grid, dim3(SP_THREADS), split_dc_lds_bytes(n, S), s, n, K, basis,
                       enc, P, Gs, N, Np, X, sig_w, dC);
    tl.done(s);
}

template <int S>
void launch_split_gemm(int64_t K, const unsigned short *Cts, int64_t nc, int64_t RBn, int64_t cb0,
                       const unsigned short *Gts, int64_t Pp, double *Wc, int64_t ldw, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_split_gemm<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    const dim3 grid((unsigned)ceil_div(nc, SP_BN), (unsigned)ceil_div(K, SP_BM));
    hipLaunchKernelGGL((k_split_gemm<S>), grid, dim3(SP_THREADS), split_gemm_lds_bytes(S), s, K, ceil_div(K, 32),
                       Cts, nc, RBn, cb0, Gts, Pp, Wc, ldw);
}

template <int S>
void launch_bwd_dc_split(int n, int64_t K, const uint8_t *basis, const uint4 *enc, int64_t P,
                         const unsigned short *Gs, int64_t N, int64_t Np, const double *X, const int32_t *sig_w,
                         double *dC, hipStream_t s)
{
    if (n * SP_KS <= 2 * SP_THREADS) launch_bwd_dc_split_xr<S, 2>(n, K, basis, enc, P, Gs, N, Np, X, sig_w, dC, s);
    else launch_bwd_dc_split_xr<S, 4>(n, K, basis, enc, P, Gs, N, Np, X, sig_w, dC, s);
}

}  // namespace

poly_status dense_bwd_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t S,
                                size_t *ws_bytes)
{
    if (!ws_bytes || n < 1 || n > 255 || K < 0 || P < 0 || N < 0) return POLY_ERR_ARG;
    if (prec != POLY_FP64 && prec != POLY_SPLIT_BF16) return POLY_ERR_ARG;
    if (prec == POLY_SPLIT_BF16 && (S < 3 || S > 5)) return POLY_ERR_ARG;
    *ws_bytes = plan_dense_bwd(n, K, P, N, prec, S).total;
    return POLY_OK;
}

poly_status dense_bwd_run(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P, const double *C,
                          int64_t N, const double *X, const double *gY, double *dC, double *dX, poly_prec prec,
                          int32_t S, void *ws, size_t ws_bytes, hipStream_t s)
{
    size_t need = 0;
    poly_status st = dense_bwd_workspace(n, K, P, N, prec, S, &need);
    if (st != POLY_OK) return st;
    if (max_exp < 0 || max_exp > 255) return POLY_ERR_ARG;
    if ((K > 0 && !basis) || (P > 0 && K > 0 && !C) || (N > 0 && !X) || (P > 0 && N > 0 && !gY)) return POLY_ERR_ARG;
    if (!ws || ws_bytes < need) return POLY_ERR_WORKSPACE;
    if (dX && dense_bwd_dx_lds(n) > DB_DX_LDS_MAX) return POLY_ERR_UNSUPPORTED;
    const DenseBwdPlan d = plan_dense_bwd(n, K, P, N, prec, S);
    // split dC: a step's coordinates are at most SW_XR_MAX per thread (n <= 64),
    // and a workgroup's rows of one gY plane stay below 2^31 bytes
    if (prec == POLY_SPLIT_BF16 && dC &&
        ((int64_t)n * SP_KS > (int64_t)SW_XR_MAX * SP_THREADS || split_dc_lds_bytes(n, S) > 160 * 1024 ||
         d.Np * 512 + 256 > INT32_MAX))
        return POLY_ERR_UNSUPPORTED;
    // split dX: a workgroup's rows of one C^T plane below 2^31 bytes
    if (prec == POLY_SPLIT_BF16 && dX && d.Pp * 512 + 256 > INT32_MAX) return POLY_ERR_UNSUPPORTED;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_dense_bwd_dx, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)DB_DX_LDS_MAX);
        (void)hipFuncSetAttribute((const void *)k_dense_bwd_dc<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  64 * 1024);
        (void)hipFuncSetAttribute((const void *)k_dense_bwd_dc<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  64 * 1024);
        attr = true;
    }
    uint4 *fenc = (uint4 *)((char *)ws + d.fenc);
    uint64_t *senc = (uint64_t *)((char *)ws + d.senc);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)ws, 0ull, (int64_t)1);
    if (K > 0) {
        hipLaunchKernelGGL(k_encode_factors, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, basis, K, n,
                           (uint32_t *)fenc, (const int64_t *)nullptr, (uint32_t *)nullptr);
        hipLaunchKernelGGL(k_encode_support, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, basis, K, n, senc,
                           (const int64_t *)nullptr);
    }
    if (dC && P > 0 && K > 0) {
        if (N == 0) {
            hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<int64_t>(ceil_div(P * K, 256), 65535)), dim3(256), 0, s,
                               (unsigned long long *)dC, 0ull, P * K);
        } else if (prec == POLY_SPLIT_BF16) {
            unsigned short *Gs = (unsigned short *)((char *)ws + d.gs);
            int32_t *sig_w = (int32_t *)((char *)ws + d.sigw);
            const int64_t npb = ceil_div(N, DN_KB);
            static bool wattr = false;
            if (!wattr) {
                (void)hipFuncSetAttribute((const void *)k_split_wscale, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          160 * 1024);
                wattr = true;
            }
            hipLaunchKernelGGL(k_split_c, dim3((unsigned)(ceil_div(P, 32) * 32 * ceil_div(d.Np, DN_KB))), dim3(DN_KB),
                               0, s, gY, P, N, d.Np, S, Gs);
            hipLaunchKernelGGL(k_split_wscale, dim3((unsigned)(npb * ceil_div(K, 256))), dim3(256),
                               (size_t)DN_KB * (n + 1) * 8, s, n, K, basis, (const uint4 *)fenc, N, X, sig_w);
            switch (S) {
            case 3: launch_bwd_dc_split<3>(n, K, basis, fenc, P, Gs, N, d.Np, X, sig_w, dC, s); break;
            case 4: launch_bwd_dc_split<4>(n, K, basis, fenc, P, Gs, N, d.Np, X, sig_w, dC, s); break;
            default: launch_bwd_dc_split<5>(n, K, basis, fenc, P, Gs, N, d.Np, X, sig_w, dC, s); break;
            }
        } else {
            const int bm = tunables().dense_f64_rows == 128 ? 128 : 64;
            const dim3 grid((unsigned)ceil_div(K, DB_BN), (unsigned)ceil_div(P, bm));
            TimedLaunch tl(POLY_TIMING_DENSE, s);
            if (bm == 128)
                hipLaunchKernelGGL(k_dense_bwd_dc<128>, grid, dim3(DB_THREADS), (size_t)(n + 1) * DB_KS * 8, s, n, K,
                                   basis, (const uint4 *)fenc, P, gY, N, X, dC);
            else
                hipLaunchKernelGGL(k_dense_bwd_dc<64>, grid, dim3(DB_THREADS), (size_t)(n + 1) * DB_KS * 8, s, n, K,
                                   basis, (const uint4 *)fenc, P, gY, N, X, dC);
            tl.done(s);
        }
    }
    if (dX && N > 0 && prec == POLY_SPLIT_BF16 && P > 0 && K > 0) {
        unsigned short *Cts = (unsigned short *)((char *)ws + d.ct);
        unsigned short *Gts = (unsigned short *)((char *)ws + d.gyt);
        double *Wc = (double *)((char *)ws + d.w);
        double *part = (double *)((char *)ws + d.part);
        static bool xattr = false;
        if (!xattr) {
            (void)hipFuncSetAttribute((const void *)k_dx_from_w, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      160 * 1024);
            xattr = true;
        }
        const int64_t nkb = ceil_div(d.Pp, DN_KB);
        hipLaunchKernelGGL(k_split_ct, dim3((unsigned)(ceil_div(K, 32) * nkb)), dim3(DN_KB), 0, s, C, K, K, P, d.Pp,
                           S, Cts);
        hipLaunchKernelGGL(k_split_ct, dim3((unsigned)(ceil_div(N, 32) * nkb)), dim3(DN_KB), 0, s, gY, N, N, P, d.Pp,
                           S, Gts);
        const size_t xlds = ((size_t)(n + 1) * 64 + (size_t)DW_WAVES * n * 64) * 8;
        for (int64_t c0 = 0; c0 < N; c0 += d.Nc) {
            const int64_t nc = std::min<int64_t>(d.Nc, N - c0);
            switch (S) {
            case 3: launch_split_gemm<3>(K, Cts, nc, ceil_div(N, 32), c0 / 32, Gts, d.Pp, Wc, d.Nc, s); break;
            case 4: launch_split_gemm<4>(K, Cts, nc, ceil_div(N, 32), c0 / 32, Gts, d.Pp, Wc, d.Nc, s); break;
            default: launch_split_gemm<5>(K, Cts, nc, ceil_div(N, 32), c0 / 32, Gts, d.Pp, Wc, d.Nc, s); break;
            }
            hipLaunchKernelGGL(k_dx_from_w, dim3((unsigned)ceil_div(nc, 64), (unsigned)DW_KSPLIT),
                               dim3(DW_WAVES * 64), xlds, s, n, K, basis, (const uint64_t *)senc,
                               (const double *)Wc, d.Nc, nc, X + c0 * n, part);
            hipLaunchKernelGGL(k_dx_reduce, dim3((unsigned)std::min<int64_t>(ceil_div(nc * n, 256), 65535)),
                               dim3(256), 0, s, (const double *)part, nc, n, dX + c0 * n);
        }
    } else if (dX && N > 0) {
        hipLaunchKernelGGL(k_dense_bwd_dx, dim3((unsigned)ceil_div(N, DB_BN)), dim3(DB_THREADS), dense_bwd_dx_lds(n), s,
                           n, K, basis, (const uint64_t *)senc, P, C, gY, N, X, dX);
    }
    return hipGetLastError() == hipSuccess ? POLY_OK : POLY_ERR_HIP;
}

// ------------------------------------------- CSR batches over a shared basis

// Status POLY_ERR_UNSUPPORTED unless every polynomial of the batch (P rows
// of K terms each) lists the same exponent rows as polynomial 0.
__global__ void k_check_shared(const uint8_t *exps, int64_t P, int64_t K, int n, int32_t *status)
{
    const int64_t bytes = K * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (P - 1) * bytes;
         i += (int64_t)gridDim.x * blockDim.x)
        if (exps[bytes + i] != exps[i % bytes]) {
            set_status(status, POLY_ERR_UNSUPPORTED);
            break;
        }
}

// Derived basis and coefficients of a derivative of a shared-basis batch:
// with j >= 0 (and k >= 0 for a second derivative) the basis row e becomes
// e - u_j (- u_k) and the coefficients are scaled by the integer
// multiplier m = e_j (or e_j (e_k - [j == k]), formed first), so that the
// derivative is the contraction of C' = m C with the derived monomials.  A
// row whose multiplier is zero keeps e with coefficient 0.
__global__ void k_derive_basis(const uint8_t *basis, int64_t K, int n, int j, int k, uint8_t *dbasis, const double *C,
                               int64_t P, double *dC)
{
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < P * K;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kk = idx % K;
        const uint8_t *row = basis + kk * n;
        const int ej = row[j];
        const int m = k < 0 ? ej : ej * ((int)row[k] - (k == j ? 1 : 0));
        dC[idx] = m > 0 ? C[idx] * (double)m : 0.0;
        if (idx < K) {
            for (int i = 0; i < n; ++i) {
                const int e = row[i];
                dbasis[kk * n + i] = (uint8_t)(m > 0 ? e - (i == j) - (k >= 0 && i == k) : e);
            }
        }
    }
}

// H[p][pt][k][j] = H[p][pt][j][k] for j < k (the upper triangle was written)
__global__ void k_hess_mirror(double *H, int64_t PN, int n)
{
    const int64_t total = PN * n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = idx / ((int64_t)n * n);
        const int r = (int)(idx % ((int64_t)n * n));
        const int a = r / n, b = r % n;
        if (a > b) H[idx] = H[q * n * n + (int64_t)b * n + a];
    }
}

}  // namespace polyhip
