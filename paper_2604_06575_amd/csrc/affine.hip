// Affine-normal direction of one polynomial at a batch of points (Section 5,
// the exact log-determinant route).
//
// At a point x with g = grad f(x), e = g / |g| and an orthonormal frame
// Q = [Q_T, e], the direction is nu = Q [tau; -1] with
//   A   = Q_T' H Q_T + reg I          (regularized tangent block, H = Hess f(x))
//   a_i = tr(A^-1 Q_T' D^3f[Q_T e_i] Q_T)
//   tau = A^-1 (Q_T' H e - |g| / (n + 1) a).
// With M = Q_T A^-1 Q_T' (n x n) the correction needs no third-order tensor:
// a = Q_T' w with w_l = sum_jk M_jk d^3 f / dx_j dx_k dx_l (x), and since
// Q_T' e = 0,
//   nu = M (H e - |g| / (n + 1) w) - e.
// Q_T is taken from the Householder reflector P = I - beta v v' that maps e
// to -s e_n (s the sign of e_n): its first n - 1 columns are orthonormal and
// orthogonal to e, so A is the leading block of P H P (a rank-two update of
// H) and M = P [A^-1 0; 0 0] P (another one).  The direction does not depend
// on the choice of Q_T.
//
// One workgroup per point; H (from the Hessian path), then the tangent
// block, its inverse (Gauss-Jordan with partial pivoting) and M live in LDS
// in place for n <= AN_MAX_N_LDS, and in the point's own Hessian slot in
// global memory (row stride n, kept coherent within the workgroup by its
// barriers) beyond that.  w is accumulated term by term from each monomial's factor list
// (variables in ascending order, degree <= EV_MAX_DEG) with per-point power
// tables.
#include <limits.h>

#include "kernels.h"

namespace polyhip {

namespace {

__device__ inline double readlane_d(double v, int lane)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int THREADS>
__device__ inline double block_sum_d(double v, double *scratch)
{
    double tot;
    (void)block_exclusive_scan<THREADS>(v, scratch, tot);
    return tot;
}

}  // namespace

__global__ void __launch_bounds__(AN_THREADS) k_affine_normal(int n, const uint4 *enc, const double *coefs, int64_t T,
                                                             const double *X, const double *G, double *H,
                                                             double reg, double *D, double *gnorm, int32_t *status)
{
    extern __shared__ double s_dyn[];
    const bool in_lds = n <= AN_MAX_N_LDS;
    const int ld = in_lds ? n + 1 : n;            // row stride of the matrix (padded in LDS)
    constexpr int KP = EV_MAX_DEG + 1;            // powers x^0 .. x^EV_MAX_DEG
    double *Hp = H + (size_t)blockIdx.x * n * n;
    double *S = in_lds ? s_dyn : Hp;              // [n][ld]
    double *e = in_lds ? S + (size_t)n * ld : s_dyn;   // [n] unit gradient
    double *v = e + n;                            // [n] Householder vector
    double *t = v + n;                            // [n] H v, then K v
    double *u = t + n;                            // [n] v' K
    double *he = u + n;                           // [n] H e
    double *w = he + n;                           // [n] third-derivative contraction
    double *col = w + n;                          // [n] pivot column
    double *xp = col + n;                         // [n][KP] powers
    __shared__ double s_red[AN_THREADS / kWave];
    __shared__ int s_piv[AN_MAX_N];
    __shared__ int s_kinv[kWave];
    __shared__ int s_ip;
    __shared__ double s_rowbuf[2][AN_THREADS / kWave][kWave];
    __shared__ double s_cval[2][AN_THREADS / kWave];
    __shared__ int s_crow[2][AN_THREADS / kWave];
    const int tid = threadIdx.x;
    // matrix loops: rows by wave, columns by lane (no index division)
    const int ty = tid / kWave, tx = tid % kWave;
    constexpr int NW = AN_THREADS / kWave;
    const int64_t pt = blockIdx.x;
    const int m = n - 1;
    if (in_lds)
        for (int i = ty; i < n; i += NW)
            for (int j = tx; j < n; j += kWave) S[i * ld + j] = Hp[i * n + j];
    for (int i = tid; i < n; i += AN_THREADS) {
        const double xi = X[pt * n + i];
        double p = 1.0;
        for (int k = 0; k < KP; ++k) {
            xp[i * KP + k] = p;
            p = p * xi;
        }
        e[i] = G[pt * n + i];
        w[i] = 0.0;
    }
    __syncthreads();
    double part = 0.0;
    for (int i = tid; i < n; i += AN_THREADS) part += e[i] * e[i];
    const double gn = sqrt(block_sum_d<AN_THREADS>(part, s_red));
    const double sgn = e[m] / gn >= 0.0 ? 1.0 : -1.0;
    for (int i = tid; i < n; i += AN_THREADS) {
        const double ei = e[i] / gn;
        v[i] = i == m ? ei + sgn : ei;
    }
    __syncthreads();
    for (int i = tid; i < n; i += AN_THREADS) e[i] = e[i] / gn;
    // H e and H v from the untouched Hessian
    for (int i = tid; i < n; i += AN_THREADS) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < n; ++j) {
            const double hij = S[i * ld + j];
            a += hij * (j == m ? v[j] - sgn : v[j]);
            b += hij * v[j];
        }
        he[i] = a;
        t[i] = b;
    }
    __syncthreads();
    part = 0.0;
    for (int i = tid; i < n; i += AN_THREADS) part += v[i] * v[i];
    const double vv = block_sum_d<AN_THREADS>(part, s_red);
    part = 0.0;
    for (int i = tid; i < n; i += AN_THREADS) part += v[i] * t[i];
    const double vhv = block_sum_d<AN_THREADS>(part, s_red);
    const double beta = 2.0 / vv;
    // P H P = H - beta (v t' + t v') + beta^2 (v'Hv) v v', in place; then the
    // regularized tangent block A in the leading (n-1) x (n-1) corner
    for (int i = ty; i < n; i += NW)
        for (int j = tx; j < n; j += kWave) {
            double b = S[i * ld + j] - beta * (v[i] * t[j] + t[i] * v[j]) + beta * beta * vhv * v[i] * v[j];
            if (i == j && i < m) b += reg;
            S[i * ld + j] = b;
        }
    __syncthreads();
    // ---- A^-1 in place: Gauss-Jordan with partial (row) pivoting
    if (m <= kWave) {
        // Register-resident for n <= 65: lane tx holds column tx of rows
        // ty, ty + NW, ... (RPT rows).  Rows are not swapped: each step's
        // pivot is the unused row with the largest entry in column k (the
        // smallest row index on ties).  Every wave offers its best row in LDS
        // (double-buffered by step parity, so one barrier per step), and the
        // column-k multipliers come from lane k by readlane.  Afterwards the
        // entry in row i, column j belongs at (kinv[i], piv[j]) of the inverse,
        // where row i was the pivot of step kinv[i] and piv[j] the pivot row of
        // step j.
        constexpr int RPT = kWave / NW;
        double a[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = ty + NW * r;
            a[r] = (i < m && tx < m) ? S[i * ld + tx] : 0.0;
        }
        uint64_t used = 0;
        for (int k = 0; k < m; ++k) {
            const int par = k & 1;
            // this wave's candidate (computed on every lane, lane k's counts)
            double bv = -1.0;
            int br = -1;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = ty + NW * r;
                const double v = fabs(a[r]);
                if (i < m && !((used >> i) & 1ull) && (br < 0 || v > bv)) {
                    bv = v;
                    br = r;
                }
            }
            bv = readlane_d(bv, k);
            br = __builtin_amdgcn_readlane(br, k);
            if (br >= 0) {
                double v = a[0];
#pragma unroll
                for (int r = 1; r < RPT; ++r) v = r == br ? a[r] : v;
                s_rowbuf[par][ty][tx] = v;
            }
            if (tx == 0) {
                s_cval[par][ty] = bv;
                s_crow[par][ty] = br >= 0 ? ty + NW * br : INT_MAX;
            }
            __syncthreads();
            double best = -1.0;
            int ip = INT_MAX, wsel = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const double c = s_cval[par][w];
                const int ci = s_crow[par][w];
                if (ci == INT_MAX) continue;
                if (ip == INT_MAX || c > best || (c == best && ci < ip)) {
                    best = c;
                    ip = ci;
                    wsel = w;
                }
            }
            used |= 1ull << ip;
            const double pinv = 1.0 / s_rowbuf[par][wsel][k];
            const double pl = s_rowbuf[par][wsel][tx] * pinv;   // scaled pivot row, column tx
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = ty + NW * r;
                if (i == ip) {
                    a[r] = tx == k ? pinv : pl;
                } else {
                    const double c = readlane_d(a[r], k);
                    a[r] = tx == k ? -c * pinv : a[r] - c * pl;
                }
            }
            if (tid == 0) {
                s_piv[k] = ip;
                s_kinv[ip] = k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = ty + NW * r;
            if (i < m && tx < m) S[s_kinv[i] * ld + s_piv[tx]] = a[r];
        }
        __syncthreads();
    } else {
        // larger n: the matrix stays in LDS, rows swapped, swaps undone after
        for (int k = 0; k < m; ++k) {
            if (tid < kWave) {
                double best = -1.0;
                int bi = k;
                for (int i = k + tid; i < m; i += kWave) {
                    const double a = fabs(S[i * ld + k]);
                    if (a > best) {
                        best = a;
                        bi = i;
                    }
                }
    #pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) {
                    const double ob = __shfl_xor(best, o, kWave);
                    const int oi = __shfl_xor(bi, o, kWave);
                    if (ob > best || (ob == best && oi < bi)) {
                        best = ob;
                        bi = oi;
                    }
                }
                if (tid == 0) {
                    s_ip = bi;
                    s_piv[k] = bi;
                }
            }
            __syncthreads();
            const int ip = s_ip;
            if (ip != k)
                for (int j = tid; j < m; j += AN_THREADS) {
                    const double a = S[k * ld + j];
                    S[k * ld + j] = S[ip * ld + j];
                    S[ip * ld + j] = a;
                }
            __syncthreads();
            const double pinv = 1.0 / S[k * ld + k];
            for (int i = tid; i < m; i += AN_THREADS) col[i] = S[i * ld + k];
            __syncthreads();
            for (int j = tid; j < m; j += AN_THREADS) S[k * ld + j] = j == k ? pinv : S[k * ld + j] * pinv;
            __syncthreads();
            for (int i = ty; i < m; i += NW) {
                if (i == k) continue;
                const double ci = col[i];
                for (int j = tx; j < m; j += kWave)
                    S[i * ld + j] = j == k ? -ci * pinv : S[i * ld + j] - ci * S[k * ld + j];
            }
            __syncthreads();
        }
        for (int k = m - 1; k >= 0; --k) {   // undo the row swaps as column swaps, last first
            const int ip = s_piv[k];
            if (ip != k)
                for (int i = tid; i < m; i += AN_THREADS) {
                    const double a = S[i * ld + k];
                    S[i * ld + k] = S[i * ld + ip];
                    S[i * ld + ip] = a;
                }
            __syncthreads();
        }
    }
    // ---- M = P K P with K = [A^-1 0; 0 0]
    for (int i = tid; i < n; i += AN_THREADS) {
        S[m * ld + i] = 0.0;
        S[i * ld + m] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += AN_THREADS) {
        double kv = 0.0, vk = 0.0;
        for (int j = 0; j < n; ++j) {
            kv += S[i * ld + j] * v[j];
            vk += v[j] * S[j * ld + i];
        }
        t[i] = kv;
        u[i] = vk;
    }
    __syncthreads();
    part = 0.0;
    for (int i = tid; i < n; i += AN_THREADS) part += v[i] * t[i];
    const double vkv = block_sum_d<AN_THREADS>(part, s_red);
    for (int i = ty; i < n; i += NW)
        for (int j = tx; j < n; j += kWave)
            S[i * ld + j] = S[i * ld + j] - beta * (t[i] * v[j] + v[i] * u[j]) + beta * beta * vkv * v[i] * v[j];
    __syncthreads();
    // ---- w_l = sum_jk M_jk f_jkl(x), term by term
    for (int64_t q = tid; q < T; q += AN_THREADS) {
        const uint4 f = enc[q];
        const int d = (int)f.w;
        if (d > EV_MAX_DEG) {
            set_status(status, POLY_ERR_UNSUPPORTED);
            continue;
        }
        if (d < 3) continue;
        const uint32_t words[3] = {f.x, f.y, f.z};
        int var[EV_MAX_DEG], mul[EV_MAX_DEG];
        int s = 0;
        for (int r = 0; r < d; ++r) {
            const int vi = (int)((words[r >> 2] >> (8 * (r & 3))) & 0xffu);
            if (s > 0 && var[s - 1] == vi) {
                ++mul[s - 1];
            } else {
                var[s] = vi;
                mul[s] = 1;
                ++s;
            }
        }
        const double c = coefs[q];
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b) {
                const int kb = mul[b] - (a == b);
                if (mul[a] <= 0 || kb <= 0) continue;
                const double mab = S[var[a] * ld + var[b]];
                for (int l = 0; l < s; ++l) {
                    const int kl = mul[l] - (a == l) - (b == l);
                    if (kl <= 0) continue;
                    double val = c * (double)(mul[a] * kb * kl) * mab;
                    for (int r = 0; r < s; ++r)
                        val *= xp[var[r] * KP + (mul[r] - (a == r) - (b == r) - (l == r))];
                    atomicAdd(&w[var[l]], val);
                }
            }
    }
    __syncthreads();
    // ---- nu = M (H e - |g| / (n + 1) w) - e
    const double cg = gn / (double)(n + 1);
    for (int i = tid; i < n; i += AN_THREADS) col[i] = he[i] - cg * w[i];
    __syncthreads();
    for (int i = tid; i < n; i += AN_THREADS) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += S[i * ld + j] * col[j];
        D[pt * n + i] = r - e[i];
    }
    if (gnorm && tid == 0) gnorm[pt] = gn;
}

}  // namespace polyhip
