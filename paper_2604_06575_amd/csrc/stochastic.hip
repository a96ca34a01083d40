// Affine-normal direction of one polynomial at a batch of points by the
// stochastic log-determinant route of Section 5 (MF-logDet-Stochastic).
//
// The exact route needs the traces a_i = tr(A^-1 d_{t_i} H_T) of the
// regularized tangent block A = Q_T' H Q_T + reg I.  Here each trace is a
// Hutchinson average over q probes and every solve with A is a Krylov
// (conjugate-gradient) solve, so neither H nor A is ever formed: the method
// needs Hessian-vector products and third-derivative contractions, both
// taken term by term from the monomials.
//
// The iteration runs in R^n on the tangent space e-perp (e = g / |g|)
// instead of in the coordinates of a tangent frame: with P = I - e e', the
// operator A~ v = P H P v + reg P v is Q_T A Q_T' on e-perp, a probe Z_s
// (given in R^n) has the tangent part v_s = P Z_s = Q_T (Q_T' Z_s), and
// conjugate gradients are invariant under the isometry Q_T, so the iterates
// are Q_T times those of the frame coordinates and no frame is built.  The
// residual is projected onto e-perp after every step and A~ is zero on e,
// so the iterates never solve for rounding-level e-components (with
// P H v + reg v, e would be an eigenvector of eigenvalue reg and such
// components would grow by 1/reg; without the projection they would come to
// dominate the search direction once the tangent part has converged).
//   y_s = A~^-1 v_s                     (conjugate gradients per probe)
//   w   = (1/q) sum_s D^3 f[y_s, v_s, .]
//   tau = A~^-1 P (H e - |g| / (n + 1) w)    (one more solve)
//   nu  = tau - e.
// Conjugate gradients start from 0 and take a step (one product A~ p) while
// fewer than maxit products have been made and |r| > tol |b|; p'A~p = 0
// ends the solve.
//
// Derivatives of a monomial come from its factor list (one entry per unit
// of degree, variables ascending): m(x) = prod_r x_{v_r}, so
// d m / dx_j = sum_{r: v_r = j} prod_{r' != r} x_{v_r'}.  Evaluating the
// products on x + eps u (eps^2 = 0) gives the Hessian-vector product as the
// eps part, and on x + eps1 u + eps2 v (eps1^2 = eps2^2 = 0) the contraction
// D^3 m[u, v, .] as the eps1 eps2 part: prefix and suffix products of the
// truncated factors, no powers, no division, exact at zero coordinates.
//
// One workgroup per point.  Probes are solved B at a time (B a power of two
// dividing the workgroup), each by a group of 256 / B threads that own the
// probe's vector entries: reductions stay inside the group (lane shuffles,
// plus LDS across waves when a group spans waves), the per-probe scalars live
// in registers, and the only cross-group steps are the term passes, which
// take (term, probe) pairs.  Everything lives in LDS:
//   x, e, H e, w            [n] each
//   V, Y, R, Pv, AP         [B][n] each (probe, solution, residual,
//                                        direction, product accumulator)
#include "kernels.h"

namespace polyhip {

namespace {

struct Dual1 {
    double a, b;
};
struct Dual2 {
    double a, b, c, d;
};

__device__ inline double mul(double x, double y) { return x * y; }
__device__ inline Dual1 mul(Dual1 x, Dual1 y) { return {x.a * y.a, x.a * y.b + x.b * y.a}; }
__device__ inline Dual2 mul(Dual2 x, Dual2 y)
{
    return {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a, x.a * y.d + x.d * y.a + x.b * y.c + x.c * y.b};
}
__device__ inline double top(double x) { return x; }
__device__ inline double top(Dual1 x) { return x.b; }
__device__ inline double top(Dual2 x) { return x.d; }
template <class T>
__device__ inline T one();
template <>
__device__ inline double one<double>() { return 1.0; }
template <>
__device__ inline Dual1 one<Dual1>() { return {1.0, 0.0}; }
template <>
__device__ inline Dual2 one<Dual2>() { return {1.0, 0.0, 0.0, 0.0}; }

__device__ inline double factor(const double *x, const double *, const double *, int i, double) { return x[i]; }
__device__ inline Dual1 factor(const double *x, const double *u, const double *, int i, Dual1)
{
    return {x[i], u[i]};
}
__device__ inline Dual2 factor(const double *x, const double *u, const double *v, int i, Dual2)
{
    return {x[i], u[i], v[i], 0.0};
}

// out[j] += c * top(d/dx_j prod_r L_r) for one monomial's factor list,
// L_r = x_{v_r} (+ eps u_{v_r} (+ eps2 v_{v_r})).  Returns false for a
// degree above EV_MAX_DEG.
template <class T>
__device__ inline bool term_pass(uint4 f, double c, const double *x, const double *u, const double *v, double *out)
{
    const int d = (int)f.w;
    if (d > EV_MAX_DEG) return false;
    const uint32_t words[3] = {f.x, f.y, f.z};
    int var[EV_MAX_DEG];
    T suf[EV_MAX_DEG + 1];
#pragma unroll
    for (int r = 0; r < EV_MAX_DEG; ++r) var[r] = (int)((words[r >> 2] >> (8 * (r & 3))) & 0xffu);
#pragma unroll
    for (int r = 0; r <= EV_MAX_DEG; ++r) suf[r] = one<T>();
#pragma unroll
    for (int r = EV_MAX_DEG - 1; r >= 0; --r)
        if (r < d) suf[r] = mul(factor(x, u, v, var[r], T{}), suf[r + 1]);
    T pre = one<T>();
    double run = 0.0;
#pragma unroll
    for (int r = 0; r < EV_MAX_DEG; ++r) {
        if (r < d) {
            run += top(mul(pre, suf[r + 1]));
            // the factor list is sorted: flush at the last occurrence of a variable
            if (r + 1 == d || var[r + 1] != var[r]) {
                atomicAdd(&out[var[r]], c * run);
                run = 0.0;
            }
            pre = mul(pre, factor(x, u, v, var[r], T{}));
        }
    }
    return true;
}

// Sum of NV values over the G threads of a probe group (G a power of two,
// groups aligned); every thread of the block calls it with the same G.
// Every thread of a group receives the same bits (a butterfly of commutative
// additions, then one fixed order across waves).
template <int NV>
__device__ inline void group_sum(double (&v)[NV], int G, double *s_red)
{
    const int width = G < kWave ? G : kWave;
    for (int off = width >> 1; off > 0; off >>= 1)
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] += __shfl_xor(v[j], off, kWave);
    if (G > kWave) {
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        __syncthreads();
        if (lane == 0)
#pragma unroll
            for (int j = 0; j < NV; ++j) s_red[wave * NV + j] = v[j];
        __syncthreads();
        const int gw = G / kWave, first = wave / gw * gw;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double t = 0.0;
            for (int k = 0; k < gw; ++k) t += s_red[(first + k) * NV + j];
            v[j] = t;
        }
    }
}

}  // namespace

__global__ void __launch_bounds__(AS_THREADS) k_affine_stochastic(AffStochArgs A)
{
    extern __shared__ double s_dyn[];
    __shared__ double s_red[(AS_THREADS / kWave) * 4];
    __shared__ int s_act[AS_MAX_SLOTS];
    __shared__ int s_hv;
    const int n = A.n, B = A.slots, G = AS_THREADS / B;
    const int tid = threadIdx.x, slot = tid / G, sub = tid % G;
    const int64_t pt = blockIdx.x;
    double *x = s_dyn, *e = x + n, *he = e + n, *w = he + n;
    double *V = w + n, *Y = V + (size_t)B * n, *R = Y + (size_t)B * n, *Pv = R + (size_t)B * n,
           *AP = Pv + (size_t)B * n;
    double *v_s = V + (size_t)slot * n, *y_s = Y + (size_t)slot * n, *r_s = R + (size_t)slot * n,
           *p_s = Pv + (size_t)slot * n, *ap_s = AP + (size_t)slot * n;
    const uint4 *enc = A.enc;
    const double *coefs = A.coefs;
    const int64_t T = A.T;

    for (int i = tid; i < n; i += AS_THREADS) {
        x[i] = A.X[pt * n + i];
        e[i] = 0.0;
        he[i] = 0.0;
        w[i] = 0.0;
    }
    for (int i = tid; i < B * n; i += AS_THREADS) AP[i] = 0.0;
    if (tid == 0) s_hv = 1;   // the product H e
    __syncthreads();
    // ---- gradient, then e = g / |g| and H e
    bool bad = false;
    for (int64_t t = tid; t < T; t += AS_THREADS) bad |= !term_pass<double>(enc[t], coefs[t], x, x, x, e);
    __syncthreads();
    double part = 0.0;
    for (int i = tid; i < n; i += AS_THREADS) part += e[i] * e[i];
    const double gn = sqrt(block_sum<AS_THREADS>(part, s_red));
    for (int i = tid; i < n; i += AS_THREADS) e[i] = e[i] / gn;
    __syncthreads();
    for (int64_t t = tid; t < T; t += AS_THREADS) (void)term_pass<Dual1>(enc[t], coefs[t], x, e, x, he);
    __syncthreads();
    part = 0.0;
    for (int i = tid; i < n; i += AS_THREADS) part += e[i] * he[i];
    const double eHe = block_sum<AS_THREADS>(part, s_red);

    // Conjugate gradients on the B slots whose s_act is set; V holds the
    // right-hand sides (on e-perp), Y receives the solutions.  Every thread
    // runs it; per-slot state is in the registers of the slot's group.
    auto solve = [&](bool live) -> int {
        double rr;
        {
            double s1[1] = {0.0};
            for (int i = sub; i < n; i += G) {
                const double b = v_s[i];
                y_s[i] = 0.0;
                r_s[i] = b;
                p_s[i] = b;
                s1[0] += b * b;
            }
            group_sum<1>(s1, G, s_red);
            rr = s1[0];
        }
        const double bn = sqrt(rr);
        int k = 0;
        bool active = live && k < A.maxit && sqrt(rr) > A.tol * bn;
        if (sub == 0) s_act[slot] = active;
        while (__syncthreads_or(active)) {
            // A~ p for every active slot: (term, slot) pairs
            const int64_t pairs = T * B;
            for (int64_t idx = tid; idx < pairs; idx += AS_THREADS) {
                const int s = (int)(idx & (B - 1));
                const int64_t t = idx / B;
                if (!s_act[s]) continue;
                (void)term_pass<Dual1>(enc[t], coefs[t], x, Pv + (size_t)s * n, x, AP + (size_t)s * n);
            }
            __syncthreads();
            double s4[4] = {0.0, 0.0, 0.0, 0.0};   // e'Hp, p'Hp, e'p, p'p
            for (int i = sub; i < n; i += G) {
                const double hp = ap_s[i], pi = p_s[i], ei = e[i];
                s4[0] += ei * hp;
                s4[1] += pi * hp;
                s4[2] += ei * pi;
                s4[3] += pi * pi;
            }
            group_sum<4>(s4, G, s_red);
            // q = P H P p + reg P p; with e'p = ep (zero up to rounding) and
            // H symmetric, p'q = p'Hp - 2 ep e'Hp + ep^2 e'He + reg (p'p - ep^2)
            const double eHp = s4[0], ep = s4[2];
            double alpha = 0.0;
            if (active) {
                ++k;
                const double pq = s4[1] - 2.0 * ep * eHp + ep * ep * eHe + A.reg * (s4[3] - ep * ep);
                if (pq == 0.0)
                    active = false;
                else
                    alpha = rr / pq;
            }
            double s2[2] = {0.0, 0.0};   // r'r, e'r of the updated residual
            for (int i = sub; i < n; i += G) {
                if (active) {
                    const double pi = p_s[i];
                    const double q = ap_s[i] - ep * he[i] - e[i] * (eHp - ep * eHe) + A.reg * (pi - ep * e[i]);
                    y_s[i] = y_s[i] + alpha * pi;
                    const double ri = r_s[i] - alpha * q;
                    r_s[i] = ri;
                    s2[0] += ri * ri;
                    s2[1] += e[i] * ri;
                }
                ap_s[i] = 0.0;
            }
            group_sum<2>(s2, G, s_red);
            if (active) {
                // r <- P r: its rounding-level e-component would otherwise
                // come to dominate p once the tangent part has converged,
                // and A~ is zero on e
                const double er = s2[1];
                const double rr_new = fmax(s2[0] - er * er, 0.0);
                const double beta = rr_new / rr;
                for (int i = sub; i < n; i += G) {
                    const double ri = r_s[i] - er * e[i];
                    r_s[i] = ri;
                    p_s[i] = ri + beta * p_s[i];
                }
                rr = rr_new;
                active = k < A.maxit && sqrt(rr) > A.tol * bn;
            }
            if (sub == 0) s_act[slot] = active;
        }
        return k;
    };

    const double *Zp = A.Z + (A.per_point ? pt * (int64_t)A.q * n : 0);
    for (int b0 = 0; b0 < A.q; b0 += B) {
        const bool live = b0 + slot < A.q;
        {
            // tangent part of the probe: v = Z - e (e'Z)
            double s1[1] = {0.0};
            for (int i = sub; i < n; i += G) {
                const double z = live ? Zp[(int64_t)(b0 + slot) * n + i] : 0.0;
                v_s[i] = z;
                s1[0] += e[i] * z;
            }
            group_sum<1>(s1, G, s_red);
            for (int i = sub; i < n; i += G) v_s[i] = v_s[i] - e[i] * s1[0];
        }
        const int k = solve(live);
        if (sub == 0 && live) atomicAdd(&s_hv, k);
        // D^3 f[y_s, v_s, .] per live slot into AP, then summed into w in
        // slot order
        const int64_t pairs = T * B;
        for (int64_t idx = tid; idx < pairs; idx += AS_THREADS) {
            const int s = (int)(idx & (B - 1));
            const int64_t t = idx / B;
            if (b0 + s >= A.q) continue;
            (void)term_pass<Dual2>(enc[t], coefs[t], x, Y + (size_t)s * n, V + (size_t)s * n, AP + (size_t)s * n);
        }
        __syncthreads();
        for (int i = tid; i < n; i += AS_THREADS) {
            double acc = w[i];
            for (int s = 0; s < B; ++s) {
                acc += AP[(size_t)s * n + i];
                AP[(size_t)s * n + i] = 0.0;
            }
            w[i] = acc;
        }
        __syncthreads();
    }
    // ---- tau: the solve of P (H e - |g| / (n + 1) w) in slot 0
    const double cg = gn / (double)(n + 1);
    {
        double s1[1] = {0.0};
        for (int i = sub; i < n; i += G) {
            const double t = he[i] - cg * (w[i] / (double)A.q);
            v_s[i] = t;
            s1[0] += e[i] * t;
        }
        group_sum<1>(s1, G, s_red);
        for (int i = sub; i < n; i += G) v_s[i] = v_s[i] - e[i] * s1[0];
    }
    const int kt = solve(slot == 0);
    if (slot == 0) {
        for (int i = sub; i < n; i += G) A.D[pt * n + i] = y_s[i] - e[i];
        if (sub == 0) atomicAdd(&s_hv, kt);
    }
    if (bad) set_status(A.status, POLY_ERR_UNSUPPORTED);
    __syncthreads();
    if (tid == 0) {
        A.gnorm[pt] = gn;
        if (A.hv) A.hv[pt] = s_hv;
    }
}

}  // namespace polyhip
