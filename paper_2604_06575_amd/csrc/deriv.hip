// First and second derivatives of sparse polynomials streamed from their
// source terms (Section 3.3: diff, jacobian, eval; the reverse mode of eval
// and its own reverse mode for autograd).
//
// Points sit in lanes (64 per wave, their coordinates in an LDS tile shared
// by the workgroup); terms are streamed wave-uniformly as factor lists (the
// variable indices of a monomial with repetition, ascending, padded with the
// index of an LDS row of ones).  For factor values f_0..f_{d-1} of a term with
// coefficient c, a variable j occupying e_j consecutive positions starting at
// a has
//     d m / d x_j = e_j * prod_{i != a} f_i,
// and for two variables j != k starting at a < b
//     d^2 m / dx_j dx_k = e_j e_k * prod_{i != a, b} f_i,
//     d^2 m / dx_j^2   = e_j (e_j - 1) * prod_{i != a, a+1} f_i,
// the products over the remaining positions taken from prefix and suffix
// products of the list, so no derivative polynomial is formed or sorted.
// Per-point results that are n-vectors (gradients, dX, Hessian-vector
// products) accumulate in a wave-private LDS block [n][65] (lane = point
// column) and leave in output order with whole-wave contiguous stores.
//
// Modes:
//   DM_GRAD  G[p][pt][j]  = sum_{t in p} c_t d m_t / dx_j            (poly_grad)
//   DM_DX    dX[pt][j]    = sum_t gY[p(t)][pt] c_t d m_t / dx_j       (poly_eval_backward)
//   DM_HVP   ggX[pt][j]   = sum_t gY[p(t)][pt] (c_t sum_k u[pt][k] d2 m_t / dx_j dx_k
//                                               + w_t d m_t / dx_j)  (poly_eval_backward2)
//   DM_DIRD  ggY[p][pt]   = sum_{t in p} (c_t sum_k u[pt][k] d m_t / dx_k + w_t m_t)
// Terms of degree above EV_MAX_DEG are handled from their dense exponent row.
#include "kernels.h"

namespace polyhip {

namespace {

constexpr int DV_ACC_LD = DV_ACC_PITCH;   // accumulator row pitch: columns are read across rows without bank conflicts

__device__ inline double powi_d(double x, uint32_t e)
{
    double p = 1.0;
    for (uint32_t k = 0; k < e; ++k) p = p * x;
    return p;
}

template <int MODE>
struct ModeTraits {
    static constexpr bool acc = MODE != DM_DIRD;          // per-point n-vector result
    static constexpr bool weighted = MODE == DM_DX || MODE == DM_HVP;   // gY per polynomial
    static constexpr bool dir = MODE == DM_HVP || MODE == DM_DIRD;      // reads the direction u
};

// Contribution of one term of degree d <= NP (NP = 4, 8 or 12 list positions,
// positions >= d hold the padding index, whose value is 1.0).
template <int NP, int MODE>
__device__ inline void term_fact(const DerivArgs &A, const uint32_t wd[3], int d, double c, double w2, double wgt,
                                 const double *xl, const double *ul, double *al, double &sacc)
{
    int var[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) var[k] = (int)((wd[k >> 2] >> (8 * (k & 3))) & 0xffu);
    double f[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) f[k] = xl[var[k] * kWave];
    // run starts and lengths (uniform)
    bool st[NP];
    int e[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        st[a] = a < d && (a == 0 || var[a] != var[a - 1]);
        int cnt = 1;
#pragma unroll
        for (int b = a + 1; b < NP; ++b) cnt += (b < d && var[b] == var[a]) ? 1 : 0;
        e[a] = cnt;
    }
    double pre[NP + 1], suf[NP + 1];
    pre[0] = 1.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) pre[k + 1] = pre[k] * f[k];
    suf[NP] = 1.0;
#pragma unroll
    for (int k = NP - 1; k >= 0; --k) suf[k] = f[k] * suf[k + 1];
    if constexpr (MODE == DM_GRAD || MODE == DM_DX) {
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            if (st[a]) {
                const double v = (c * (double)e[a]) * (pre[a] * suf[a + 1]);
                double *p = al + var[a] * DV_ACC_LD;
                if constexpr (MODE == DM_GRAD) *p += v;
                else *p = __builtin_fma(wgt, v, *p);
            }
        }
    } else if constexpr (MODE == DM_DIRD) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a)
            if (st[a]) s = __builtin_fma(ul[var[a] * kWave], (double)e[a] * (pre[a] * suf[a + 1]), s);
        sacc = __builtin_fma(c, s, sacc);
        sacc = __builtin_fma(w2, pre[NP], sacc);
    } else {   // DM_HVP
        double u[NP], hv[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            u[a] = st[a] ? ul[var[a] * kWave] : 0.0;
            hv[a] = 0.0;
        }
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            if (!st[a]) continue;
            // the same variable twice: positions a and a + 1
            if (a + 1 < NP && e[a] >= 2) {
                const double h = (double)(e[a] * (e[a] - 1)) * (pre[a] * suf[a + 2]);
                hv[a] = __builtin_fma(u[a], h, hv[a]);
            }
            double mid = 1.0;   // product of positions strictly between a and b
#pragma unroll
            for (int b = a + 1; b < NP; ++b) {
                if (st[b]) {
                    const double h = (double)(e[a] * e[b]) * ((pre[a] * mid) * suf[b + 1]);
                    hv[a] = __builtin_fma(u[b], h, hv[a]);
                    hv[b] = __builtin_fma(u[a], h, hv[b]);
                }
                mid = mid * f[b];
            }
        }
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            if (st[a]) {
                double v = c * hv[a];
                v = __builtin_fma(w2 * (double)e[a], pre[a] * suf[a + 1], v);
                double *p = al + var[a] * DV_ACC_LD;
                *p = __builtin_fma(wgt, v, *p);
            }
        }
    }
}

// Terms of degree above EV_MAX_DEG: the same quantities from the dense row.
template <int MODE>
__device__ inline void term_dense(const DerivArgs &A, int64_t t, double c, double w2, double wgt, const double *xl,
                                  const double *ul, double *al, double &sacc)
{
    const int n = A.n;
    const uint8_t *row = A.exps + t * n;
    auto xv = [&](int i) { return xl[i * kWave]; };
    // product of x_i^{e_i - [i == j] - [i == k]} over the support
    auto reduced = [&](int j, int k) {
        double p = 1.0;
        for (int i = 0; i < n; ++i) {
            int ei = row[i];
            if (!ei) continue;
            ei -= (i == j) + (i == k);
            p = p * powi_d(xv(i), (uint32_t)ei);
        }
        return p;
    };
    if constexpr (MODE == DM_GRAD || MODE == DM_DX) {
        for (int j = 0; j < n; ++j) {
            const int ej = row[j];
            if (!ej) continue;
            const double v = (c * (double)ej) * reduced(j, -1);
            double *p = al + j * DV_ACC_LD;
            if constexpr (MODE == DM_GRAD) *p += v;
            else *p = __builtin_fma(wgt, v, *p);
        }
    } else if constexpr (MODE == DM_DIRD) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            const int ej = row[j];
            if (ej) s = __builtin_fma(ul[j * kWave], (double)ej * reduced(j, -1), s);
        }
        sacc = __builtin_fma(c, s, sacc);
        sacc = __builtin_fma(w2, reduced(-1, -1), sacc);
    } else {
        for (int j = 0; j < n; ++j) {
            const int ej = row[j];
            if (!ej) continue;
            double hv = 0.0;
            for (int k = 0; k < n; ++k) {
                const int ek = row[k];
                if (!ek || (k == j && ej < 2)) continue;
                const int m = k == j ? ej * (ej - 1) : ej * ek;
                hv = __builtin_fma(ul[k * kWave], (double)m * reduced(j, k), hv);
            }
            double v = c * hv;
            v = __builtin_fma(w2 * (double)ej, reduced(j, -1), v);
            double *p = al + j * DV_ACC_LD;
            *p = __builtin_fma(wgt, v, *p);
        }
    }
}

// the polynomial holding term t: largest q with rp[q] <= t (rp nondecreasing)
__device__ inline int64_t poly_of(const int64_t *rp, int64_t P, int64_t t)
{
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace

// grid: x = blocks of 64 points, y = groups of work units; blockDim = 64 * W.
// Units: DM_GRAD / DM_DIRD: (polynomial q, term segment s of S); DM_DX /
// DM_HVP: term segment s of S of all terms in order (the weight gY[p][pt]
// changes where a polynomial ends).  Each wave sums its unit's terms in order
// and writes its result (S == 1) or a partial for k_sum_slices, which adds the
// S partials in segment order: results do not depend on scheduling.
// Dynamic LDS: the point tile [(n+1)][64] (row n = ones), the direction tile
// [n][64] (DM_HVP, DM_DIRD; zeros without a direction), one accumulator block
// [n][65] per wave (DM_GRAD, DM_DX, DM_HVP).
template <int MODE>
__global__ void __launch_bounds__(512) k_deriv_terms(DerivArgs A)
{
    using TR = ModeTraits<MODE>;
    extern __shared__ double lds[];
    const int W = blockDim.x >> 6;
    const int lane = lane_id();
    const int w = wave_id();
    const int n = A.n;
    const int64_t N = A.N;
    const int64_t pt0 = (int64_t)blockIdx.x * kWave;
    const int64_t pt = pt0 + lane;
    // the direction tile (zeros when no direction is given)
    constexpr bool use_u = TR::dir;
    double *s_x = lds;
    double *s_u = lds + (n + 1) * kWave;
    double *s_acc = s_u + (use_u ? n * kWave : 0) + (size_t)w * n * DV_ACC_LD;
    for (int idx = threadIdx.x; idx < (n + 1) * kWave; idx += blockDim.x) {
        const int i = idx / kWave, l = idx % kWave;
        const int64_t p = pt0 + l;
        s_x[idx] = i == n ? 1.0 : (p < N ? A.X[p * n + i] : 0.0);
        if (use_u && i < n) s_u[idx] = (p < N && A.U) ? A.U[p * n + i] : 0.0;
    }
    if constexpr (TR::acc)
        for (int j = 0; j < n; ++j) s_acc[j * DV_ACC_LD + lane] = 0.0;
    __syncthreads();   // the only workgroup barrier: waves run independently from here
    const double *xl = s_x + lane;
    const double *ul = s_u + lane;
    double *al = s_acc + lane;
    int vz;   // a zero the compiler treats as per-lane: term records are fetched by vector loads
    asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
    const int64_t S = A.S;
    const int64_t units = TR::weighted ? S : A.P * S;
    const int64_t ustride = (int64_t)gridDim.y * W;
    const uint4 *enc = reinterpret_cast<const uint4 *>(A.enc);
    for (int64_t u = (int64_t)blockIdx.y * W + w; u < units; u += ustride) {
        int64_t q, sg, ta, tb;
        if constexpr (TR::weighted) {
            sg = u;
            ta = A.T * sg / S;
            tb = A.T * (sg + 1) / S;
            q = ta < A.T ? poly_of(A.rp, A.P, ta) : A.P - 1;
        } else {
            q = u / S;
            sg = u % S;
            const int64_t b0 = A.rp[q], b1 = A.rp[q + 1];
            const int64_t len = b1 > b0 ? b1 - b0 : 0;
            ta = b0 + len * sg / S;
            tb = b0 + len * (sg + 1) / S;
        }
        int64_t qend = A.rp[q + 1];
        double wgt = 1.0;
        if constexpr (TR::weighted) wgt = pt < N ? A.gY[q * N + pt] : 0.0;
        double sacc = 0.0;
        uint4 cw = make_uint4(0, 0, 0, 0);
        double cc = 0.0, cw2 = 0.0;
        if (ta < tb) {
            cw = enc[ta + vz];
            cc = A.coefs[ta + vz];
            if (A.coefs2) cw2 = A.coefs2[ta + vz];
        }
        for (int64_t t = ta; t < tb; ++t) {
            // next term's record in flight while this one is evaluated
            uint4 nw = cw;
            double nc = cc, nw2 = cw2;
            if (t + 1 < tb) {
                nw = enc[t + 1 + vz];
                nc = A.coefs[t + 1 + vz];
                if (A.coefs2) nw2 = A.coefs2[t + 1 + vz];
            }
            if constexpr (TR::weighted) {
                if (t >= qend) {
                    do {
                        ++q;
                        qend = A.rp[q + 1];
                    } while (t >= qend);
                    wgt = pt < N ? A.gY[q * N + pt] : 0.0;
                }
            }
            const uint32_t d = __builtin_amdgcn_readfirstlane(cw.w);
            const uint32_t wd[3] = {(uint32_t)__builtin_amdgcn_readfirstlane(cw.x),
                                    (uint32_t)__builtin_amdgcn_readfirstlane(cw.y),
                                    (uint32_t)__builtin_amdgcn_readfirstlane(cw.z)};
            const double c = cc, w2 = cw2;
            if (d == 0) {
                if constexpr (MODE == DM_DIRD) sacc += w2;   // a constant term: m = 1, no derivatives
            } else if (d <= 4) {
                term_fact<4, MODE>(A, wd, (int)d, c, w2, wgt, xl, ul, al, sacc);
            } else if (d <= 8) {
                term_fact<8, MODE>(A, wd, (int)d, c, w2, wgt, xl, ul, al, sacc);
            } else if (d <= (uint32_t)EV_MAX_DEG) {
                term_fact<EV_MAX_DEG, MODE>(A, wd, (int)d, c, w2, wgt, xl, ul, al, sacc);
            } else {
                term_dense<MODE>(A, t, c, w2, wgt, xl, ul, al, sacc);
            }
            cw = nw;
            cc = nc;
            cw2 = nw2;
        }
        // result of the unit
        if constexpr (TR::acc) {
            __builtin_amdgcn_wave_barrier();
            double *dst;
            if constexpr (TR::weighted)
                dst = S == 1 ? A.out + pt0 * n : A.partial + (sg * N + pt0) * n;
            else
                dst = S == 1 ? A.out + (q * N + pt0) * n : A.partial + ((sg * A.P + q) * N + pt0) * n;
            const int np = (int)(N - pt0 < kWave ? N - pt0 : kWave);
            const int total = np * n;
            int ptl = lane / n, j = lane - (lane / n) * n;
            for (int idx = lane; idx < total; idx += kWave) {
                dst[idx] = s_acc[j * DV_ACC_LD + ptl];
                j += kWave;
                while (j >= n) {
                    j -= n;
                    ++ptl;
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int jj = 0; jj < n; ++jj) s_acc[jj * DV_ACC_LD + lane] = 0.0;
            __builtin_amdgcn_wave_barrier();
        } else {
            if (pt < N) {
                if (S == 1) A.out[q * N + pt] = sacc;
                else A.partial[(sg * A.P + q) * N + pt] = sacc;
            }
        }
    }
}

template __global__ void k_deriv_terms<DM_GRAD>(DerivArgs);
template __global__ void k_deriv_terms<DM_DX>(DerivArgs);
template __global__ void k_deriv_terms<DM_HVP>(DerivArgs);
template __global__ void k_deriv_terms<DM_DIRD>(DerivArgs);

// out[i] = sum_{s < S} partial[s * L + i], s ascending.
__global__ void k_sum_slices(const double *partial, int64_t L, int64_t S, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    double s = partial[i];
    for (int64_t k = 1; k < S; ++k) s += partial[k * L + i];
    out[i] = s;
}

// Coefficient cotangent of the second-order reverse mode, over one chunk of
// points (lanes = terms):
//   partial[chunk][t] = sum_{pt in chunk} gY[p(t)][pt] sum_k u[pt][k] d m_t / dx_k (x_pt)
// from the support encoding (up to eight (variable, exponent) pairs; more ->
// the dense row).  Dynamic LDS: the chunk's points and directions, cp * n
// doubles each.
__global__ void __launch_bounds__(BWC_THREADS) k_backward2_dc(const int64_t *rp, int64_t P, const uint8_t *exps, int n,
                                                              int64_t T, const double *X, const double *U, int64_t N,
                                                              const double *gY, double *partial, const uint64_t *enc,
                                                              int cp)
{
    extern __shared__ double s_pts[];
    double *s_xc = s_pts;
    double *s_uc = s_pts + (size_t)cp * n;
    const int64_t c = blockIdx.y;
    const int64_t p0 = c * cp;
    const int np = (int)((N - p0) < cp ? (N - p0) : cp);
    for (int idx = threadIdx.x; idx < np * n; idx += BWC_THREADS) {
        s_xc[idx] = X[p0 * n + idx];
        s_uc[idx] = U[p0 * n + idx];
    }
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * BWC_THREADS + threadIdx.x;
    if (t >= T) return;
    const int64_t q = poly_of(rp, P, t);
    const double *g = gY + q * N + p0;
    const uint64_t w0 = enc[2 * t], w1 = enc[2 * t + 1];
    double acc = 0.0;
    if ((w0 & 0xffffull) == 0xffffull) {
        const uint8_t *row = exps + t * n;
        for (int k = 0; k < np; ++k) {
            const double *x = s_xc + k * n, *u = s_uc + k * n;
            double s = 0.0;
            for (int j = 0; j < n; ++j) {
                const int ej = row[j];
                if (!ej) continue;
                double p = 1.0;
                for (int i = 0; i < n; ++i) {
                    const int ei = row[i] - (i == j);
                    if (row[i]) p = p * powi_d(x[i], (uint32_t)ei);
                }
                s = __builtin_fma(u[j], (double)ej * p, s);
            }
            acc = __builtin_fma(g[k], s, acc);
        }
    } else {
        int var[8];
        uint32_t ex[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const uint32_t ent = (uint32_t)(((s < 4 ? w0 : w1) >> (16 * (s & 3))) & 0xffffu);
            var[s] = (int)(ent & 0xffu);
            ex[s] = ent >> 8;
        }
        for (int k = 0; k < np; ++k) {
            const double *x = s_xc + k * n, *u = s_uc + k * n;
            double pw[8], pm[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const double xv = ex[s] ? x[var[s]] : 1.0;
                pm[s] = ex[s] ? powi_d(xv, ex[s] - 1) : 1.0;
                pw[s] = ex[s] ? pm[s] * xv : 1.0;
            }
            double pre[9], suf[9];
            pre[0] = 1.0;
            suf[8] = 1.0;
#pragma unroll
            for (int s = 0; s < 8; ++s) pre[s + 1] = pre[s] * pw[s];
#pragma unroll
            for (int s = 7; s >= 0; --s) suf[s] = pw[s] * suf[s + 1];
            double dd = 0.0;
#pragma unroll
            for (int s = 0; s < 8; ++s)
                if (ex[s]) dd = __builtin_fma(u[var[s]], (double)ex[s] * ((pre[s] * pm[s]) * suf[s + 1]), dd);
            acc = __builtin_fma(g[k], dd, acc);
        }
    }
    partial[c * T + t] = acc;
}

}  // namespace polyhip
