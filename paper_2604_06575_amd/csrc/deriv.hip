// First and second derivatives of sparse polynomials streamed from their
// source terms (Section 3.3: diff, jacobian, eval; the reverse mode of eval
// and its own reverse mode for autograd).
//
// Points sit in lanes (64 per wave, their coordinates in an LDS tile shared
// by the workgroup); terms are streamed wave-uniformly in the support
// encoding: up to eight (variable, exponent) slots.  For a monomial
// m = prod_s x_{v_s}^{e_s} with p_s = x_{v_s}^{e_s} and q_s = x_{v_s}^{e_s - 1},
//     d m / dx_{v_a} = e_a q_a prod_{s != a} p_s,
//     d^2 m / dx_{v_a} dx_{v_b} = e_a e_b q_a q_b prod_{s != a, b} p_s      (a != b),
//     d^2 m / dx_{v_a}^2 = e_a (e_a - 1) x_{v_a}^{e_a - 2} prod_{s != a} p_s,
// the products over the other slots taken from prefix and suffix products,
// so no derivative polynomial is formed or sorted and the per-term
// bookkeeping is a handful of scalar instructions per slot.
// Per-point results that are n-vectors (gradients, dX, Hessian-vector
// products) accumulate in a wave-private LDS block [n][65] (lane = point
// column) by LDS adds, and leave in output order with whole-wave contiguous
// stores.
//
// Modes:
//   DM_GRAD  G[p][pt][j]  = sum_{t in p} c_t d m_t / dx_j            (poly_grad)
//   DM_DX    dX[pt][j]    = sum_t gY[p(t)][pt] c_t d m_t / dx_j       (poly_eval_backward)
//   DM_HVP   ggX[pt][j]   = sum_t gY[p(t)][pt] (c_t sum_k u[pt][k] d2 m_t / dx_j dx_k
//                                               + w_t d m_t / dx_j)  (poly_eval_backward2)
//   DM_DIRD  ggY[p][pt]   = sum_{t in p} (c_t sum_k u[pt][k] d m_t / dx_k + w_t m_t)
// Terms with more than eight variables are handled from their dense exponent row.
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

// acc += v at a wave-private LDS slot (no value returned; the LDS applies the
// adds of one wave in program order, so sums do not depend on scheduling)
__device__ inline void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Contribution of one term with at most NS (4 or 8) variables, given as
// (variable, exponent) slots in the words of its support encoding (unused
// slots are zero: exponent 0, read as x^0 = 1).  Per slot s: p_s = x^e,
// q_s = x^(e-1), r_s = x^(e-2); prefix/suffix products of the p_s give every
// product over all slots but one or two.  The coordinates of all slots are
// read from LDS before any arithmetic, so the reads overlap.
template <int NS, int MODE>
__device__ inline void term_supp(const uint32_t wd[4], double c, double w2, double wgt, const double *xl,
                                 const double *ul, double *al, double &sacc)
{
    int var[NS], ex[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const uint32_t ent = (wd[k >> 1] >> (16 * (k & 1))) & 0xffffu;
        var[k] = (int)(ent & 0xffu);
        ex[k] = (int)(ent >> 8);
    }
    double x[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) x[k] = xl[var[k] * kWave];
    double p[NS], q[NS], r[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double qq = 1.0, rr = 1.0;
        for (int i = 1; i < ex[k]; ++i) {
            rr = qq;
            qq = qq * x[k];
        }
        q[k] = qq;
        r[k] = rr;
        p[k] = ex[k] ? qq * x[k] : 1.0;
    }
    double pre[NS + 1], suf[NS + 1];
    pre[0] = 1.0;
    suf[NS] = 1.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) pre[k + 1] = pre[k] * p[k];
#pragma unroll
    for (int k = NS - 1; k >= 0; --k) suf[k] = p[k] * suf[k + 1];
    if constexpr (MODE == DM_GRAD || MODE == DM_DX) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (ex[k]) {
                const double v = (c * (double)ex[k]) * ((q[k] * pre[k]) * suf[k + 1]);
                if constexpr (MODE == DM_GRAD) lds_add(al + var[k] * DV_ACC_LD, v);
                else lds_add(al + var[k] * DV_ACC_LD, wgt * v);
            }
        }
    } else if constexpr (MODE == DM_DIRD) {
        double u[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) u[k] = ul[var[k] * kWave];
        double sd = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
            if (ex[k]) sd = __builtin_fma(u[k], (double)ex[k] * ((q[k] * pre[k]) * suf[k + 1]), sd);
        sacc = __builtin_fma(c, sd, sacc);
        sacc = __builtin_fma(w2, pre[NS], sacc);
    } else {   // DM_HVP
        double u[NS], hv[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            u[k] = ul[var[k] * kWave];
            hv[k] = 0.0;
        }
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            if (!ex[a]) continue;
            if (ex[a] >= 2) {   // d2 / dx_j^2: e (e - 1) x^(e-2) times the other slots
                const double h = (double)(ex[a] * (ex[a] - 1)) * ((r[a] * pre[a]) * suf[a + 1]);
                hv[a] = __builtin_fma(u[a], h, hv[a]);
            }
            double mid = 1.0;   // product of the slots strictly between a and b
#pragma unroll
            for (int b = a + 1; b < NS; ++b) {
                if (ex[b]) {
                    const double h = (double)(ex[a] * ex[b]) * (((q[a] * q[b]) * (pre[a] * mid)) * suf[b + 1]);
                    hv[a] = __builtin_fma(u[b], h, hv[a]);
                    hv[b] = __builtin_fma(u[a], h, hv[b]);
                }
                mid = mid * p[b];
            }
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (ex[k]) {
                double v = c * hv[k];
                v = __builtin_fma(w2 * (double)ex[k], (q[k] * pre[k]) * suf[k + 1], v);
                lds_add(al + var[k] * DV_ACC_LD, wgt * v);
            }
        }
    }
}

// Terms with more than eight variables: the same quantities from the dense row.
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
            if constexpr (MODE == DM_GRAD) lds_add(al + j * DV_ACC_LD, v);
            else lds_add(al + j * DV_ACC_LD, wgt * v);
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
            lds_add(al + j * DV_ACC_LD, wgt * v);
        }
    }
}

// value of v in lane k (k uniform)
__device__ inline double readlane_f64(double v, int k)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), k);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
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
    const int64_t S = A.S;
    const int64_t units = TR::weighted ? S : A.P * S;
    const int64_t ustride = (int64_t)gridDim.y * W;
    const uint4 *enc = reinterpret_cast<const uint4 *>(A.enc);   // support encoding, 16 bytes per term
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
        // Term records travel in groups of 64: lane l loads the record of term
        // g0 + l (one coalesced load per field), each term is then read out of
        // its lane into scalar registers, and the next group's loads are in
        // flight while the current group is evaluated.
        uint4 gw = make_uint4(0, 0, 0, 0);
        double gc = 0.0, gc2 = 0.0;
        if (ta + lane < tb) {
            gw = enc[ta + lane];
            gc = A.coefs[ta + lane];
            if (A.coefs2) gc2 = A.coefs2[ta + lane];
        }
        for (int64_t g0 = ta; g0 < tb; g0 += kWave) {
            uint4 hw = make_uint4(0, 0, 0, 0);
            double hc = 0.0, hc2 = 0.0;
            const int64_t tn = g0 + kWave + lane;
            if (tn < tb) {
                hw = enc[tn];
                hc = A.coefs[tn];
                if (A.coefs2) hc2 = A.coefs2[tn];
            }
            const int cnt = (int)(tb - g0 < kWave ? tb - g0 : kWave);
            for (int k = 0; k < cnt; ++k) {
                const int64_t t = g0 + k;
                if constexpr (TR::weighted) {
                    if (t >= qend) {
                        do {
                            ++q;
                            qend = A.rp[q + 1];
                        } while (t >= qend);
                        wgt = pt < N ? A.gY[q * N + pt] : 0.0;
                    }
                }
                const uint32_t wd[4] = {(uint32_t)__builtin_amdgcn_readlane((int)gw.x, k),
                                        (uint32_t)__builtin_amdgcn_readlane((int)gw.y, k),
                                        (uint32_t)__builtin_amdgcn_readlane((int)gw.z, k),
                                        (uint32_t)__builtin_amdgcn_readlane((int)gw.w, k)};
                const double c = readlane_f64(gc, k);
                const double w2 = A.coefs2 ? readlane_f64(gc2, k) : 0.0;
                if ((wd[0] & 0xffffu) == 0xffffu) {   // more than eight variables: the dense row
                    term_dense<MODE>(A, t, c, w2, wgt, xl, ul, al, sacc);
                } else if (wd[0] == 0) {   // a constant term: m = 1, no derivatives
                    if constexpr (MODE == DM_DIRD) sacc += w2;
                } else if ((wd[2] | wd[3]) == 0) {   // at most four variables
                    term_supp<4, MODE>(wd, c, w2, wgt, xl, ul, al, sacc);
                } else {
                    term_supp<8, MODE>(wd, c, w2, wgt, xl, ul, al, sacc);
                }
            }
            gw = hw;
            gc = hc;
            gc2 = hc2;
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
