// Symbolic derivatives and sparse term-streaming evaluation.
//
//  * diff / jacobian (Section 3.3): a term with e_j > 0 becomes
//    (e - u_j, c * e_j), order preserved.  One workgroup per entry ranks the
//    surviving terms of each variable with wavefront ballots, so the output
//    keeps storage order without any sort.
//  * Hessian entries (jacobian(jacobian(p))): the (j, k) entry, j <= k, is the
//    polynomial with coefficient c * m, m = e_j (e_k - [j == k]) formed as an
//    integer first; it is evaluated once and stored to both (j, k) and (k, j).
//  * evaluation (Section 3.3, p.eval(x0)): points in lanes, terms streamed
//    wave-uniformly.  Each term's support is pre-encoded as up to eight
//    (variable, exponent) pairs in 16 bytes, read with scalar loads; the
//    lane's point coordinates sit in LDS; x^e is formed by repeated
//    multiplication.  The waves of a workgroup share 64 points and split a
//    polynomial's terms; their partial sums are added in a fixed order.
#include "kernels.h"

namespace polyhip {

// ------------------------------------------------------------------ jacobian

__global__ void __launch_bounds__(JAC_THREADS) k_jac_count(const int64_t *rp, const uint8_t *exps, int n,
                                                           int64_t *counts)
{
    __shared__ int s_wc[JAC_THREADS / kWave][256];
    const int64_t p = blockIdx.x;
    const int64_t base = rp[p];
    const int64_t T = rp[p + 1] - base;
    const int w = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < 256; j += JAC_THREADS)
        for (int q = 0; q < JAC_THREADS / kWave; ++q) s_wc[q][j] = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < T; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const uint8_t *row = exps + (base + t) * n;
        for (int j = 0; j < n; ++j) {
            const uint32_t e = t < T ? row[j] : 0u;
            const unsigned long long m = __ballot(e > 0);
            if (lane_id() == 0) s_wc[w][j] += __popcll(m);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += JAC_THREADS) {
        int64_t c = 0;
        for (int q = 0; q < JAC_THREADS / kWave; ++q) c += s_wc[q][j];
        counts[p * n + j] = c;
    }
}

__global__ void __launch_bounds__(JAC_THREADS) k_jac_write(const int64_t *rp, const uint8_t *exps,
                                                           const double *coefs, int n, const int64_t *out_rp,
                                                           uint8_t *out_exps, double *out_coefs,
                                                           int64_t capacity, int32_t *status,
                                                           int32_t overflow_code)
{
    __shared__ int s_wc[JAC_THREADS / kWave][256];
    __shared__ int64_t s_run[256];
    const int64_t p = blockIdx.x;
    const int64_t base = rp[p];
    const int64_t T = rp[p + 1] - base;
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int j = threadIdx.x; j < n; j += JAC_THREADS) s_run[j] = out_rp[p * n + j];
    __syncthreads();
    for (int64_t c0 = 0; c0 < T; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const bool valid = t < T;
        const uint8_t *row = exps + (base + t) * n;
        for (int j = 0; j < n; ++j) {
            const uint32_t e = valid ? row[j] : 0u;
            const unsigned long long m = __ballot(e > 0);
            if (lane == 0) s_wc[w][j] = __popcll(m);
        }
        __syncthreads();
        const double c = valid ? coefs[base + t] : 0.0;
        for (int j = 0; j < n; ++j) {
            const uint32_t e = valid ? row[j] : 0u;
            const unsigned long long m = __ballot(e > 0);
            if (e > 0) {
                int64_t off = s_run[j] + __popcll(m & lt);
                for (int q = 0; q < w; ++q) off += s_wc[q][j];
                if (off < capacity) {
                    uint8_t *orow = out_exps + off * n;
                    for (int v = 0; v < n; ++v) orow[v] = row[v];
                    orow[j] = (uint8_t)(e - 1);
                    out_coefs[off] = c * (double)e;
                } else {
                    set_status(status, overflow_code);
                }
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += JAC_THREADS) {
            int64_t s = 0;
            for (int q = 0; q < JAC_THREADS / kWave; ++q) s += s_wc[q][j];
            s_run[j] += s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------- hessian

__global__ void k_pair_table(int n, uint32_t *pair_jk)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int idx = j * n - (j * (j - 1)) / 2;   // pairs before row j: sum_{r<j} (n - r)
    for (int k = j; k < n; ++k) pair_jk[idx++] = ((uint32_t)j << 16) | (uint32_t)k;
}

// Pairs [pair_base, pair_base + nb) of the pair table; the formed polynomial
// for source polynomial p and pair pair_base + q has index p * nb + q.
// grid: x = source polynomials, y = groups of HES_PAIRS_PER_BLOCK pairs.
__global__ void __launch_bounds__(JAC_THREADS) k_hes_count(const int64_t *rp, const uint8_t *exps, int n,
                                                           int64_t pair_base, int64_t nb,
                                                           const uint32_t *pair_jk, int64_t *counts)
{
    __shared__ int s_wc[JAC_THREADS / kWave][HES_PAIRS_PER_BLOCK];
    const int64_t p = blockIdx.x;
    const int64_t q0 = (int64_t)blockIdx.y * HES_PAIRS_PER_BLOCK;
    const int nq = (int)((nb - q0) < HES_PAIRS_PER_BLOCK ? (nb - q0) : HES_PAIRS_PER_BLOCK);
    const int64_t base = rp[p];
    const int64_t T = rp[p + 1] - base;
    const int w = threadIdx.x >> 6;
    for (int q = threadIdx.x; q < HES_PAIRS_PER_BLOCK; q += JAC_THREADS)
        for (int r = 0; r < JAC_THREADS / kWave; ++r) s_wc[r][q] = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < T; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const uint8_t *row = exps + (base + t) * n;
        for (int q = 0; q < nq; ++q) {
            const uint32_t jk = pair_jk[pair_base + q0 + q];
            const int j = jk >> 16, k = jk & 0xffff;
            int m = 0;
            if (t < T) m = (int)row[j] * ((int)row[k] - (j == k ? 1 : 0));
            const unsigned long long b = __ballot(m > 0);
            if (lane_id() == 0) s_wc[w][q] += __popcll(b);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += JAC_THREADS) {
        int64_t c = 0;
        for (int r = 0; r < JAC_THREADS / kWave; ++r) c += s_wc[r][q];
        counts[p * nb + q0 + q] = c;
    }
}

__global__ void __launch_bounds__(JAC_THREADS) k_hes_write(const int64_t *rp, const uint8_t *exps,
                                                           const double *coefs, int n, int64_t pair_base,
                                                           int64_t nb, const uint32_t *pair_jk,
                                                           const int64_t *out_rp, uint8_t *out_exps,
                                                           double *out_coefs, int64_t capacity, int32_t *status)
{
    __shared__ int s_wc[JAC_THREADS / kWave][HES_PAIRS_PER_BLOCK];
    __shared__ int64_t s_run[HES_PAIRS_PER_BLOCK];
    const int64_t p = blockIdx.x;
    const int64_t q0 = (int64_t)blockIdx.y * HES_PAIRS_PER_BLOCK;
    const int nq = (int)((nb - q0) < HES_PAIRS_PER_BLOCK ? (nb - q0) : HES_PAIRS_PER_BLOCK);
    const int64_t base = rp[p];
    const int64_t T = rp[p + 1] - base;
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int q = threadIdx.x; q < nq; q += JAC_THREADS) s_run[q] = out_rp[p * nb + q0 + q];
    __syncthreads();
    for (int64_t c0 = 0; c0 < T; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const bool valid = t < T;
        const uint8_t *row = exps + (base + t) * n;
        for (int q = 0; q < nq; ++q) {
            const uint32_t jk = pair_jk[pair_base + q0 + q];
            const int j = jk >> 16, k = jk & 0xffff;
            int m = 0;
            if (valid) m = (int)row[j] * ((int)row[k] - (j == k ? 1 : 0));
            const unsigned long long b = __ballot(m > 0);
            if (lane == 0) s_wc[w][q] = __popcll(b);
        }
        __syncthreads();
        const double c = valid ? coefs[base + t] : 0.0;
        for (int q = 0; q < nq; ++q) {
            const uint32_t jk = pair_jk[pair_base + q0 + q];
            const int j = jk >> 16, k = jk & 0xffff;
            int m = 0;
            if (valid) m = (int)row[j] * ((int)row[k] - (j == k ? 1 : 0));
            const unsigned long long b = __ballot(m > 0);
            if (m > 0) {
                int64_t off = s_run[q] + __popcll(b & lt);
                for (int r = 0; r < w; ++r) off += s_wc[r][q];
                if (off < capacity) {
                    uint8_t *orow = out_exps + off * n;
                    for (int v = 0; v < n; ++v) orow[v] = row[v];
                    orow[j] = (uint8_t)(orow[j] - 1);
                    orow[k] = (uint8_t)(orow[k] - 1);
                    out_coefs[off] = c * (double)m;
                } else {
                    set_status(status, POLY_ERR_WORKSPACE);
                }
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nq; q += JAC_THREADS) {
            int64_t s = 0;
            for (int r = 0; r < JAC_THREADS / kWave; ++r) s += s_wc[r][q];
            s_run[q] += s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- support encoding

// Per term: up to 8 (variable, exponent) pairs in two 64-bit words, 16 bits
// each (variable in the low byte, exponent in the high byte); unused slots are
// zero.  A term with more than eight nonzero exponents is marked 0xFFFF in the
// first slot and evaluated from its dense row.
__global__ void k_encode_support(const uint8_t *exps, int64_t T, int n, uint64_t *enc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint8_t *row = exps + t * n;
    uint64_t w[2] = {0, 0};
    int s = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t e = row[i];
        if (e == 0) continue;
        if (s < 8) w[s >> 2] |= (uint64_t)(((e << 8) | (uint32_t)i) & 0xffffu) << (16 * (s & 3));
        ++s;
    }
    if (s > 8) {
        w[0] = 0xffffull;
        w[1] = 0;
    }
    enc[2 * t] = w[0];
    enc[2 * t + 1] = w[1];
}

// ------------------------------------------------------------- evaluation

namespace {

__device__ inline double powi(double x, uint32_t e)
{
    double p = x;
    for (uint32_t k = 1; k < e; ++k) p = p * x;
    return p;
}

// Monomial value of encoded term t at the point whose coordinates are
// x[i * xs] (i = variable).
__device__ inline double term_value(const uint64_t *enc, const uint8_t *exps, int n, int64_t t, const double *x,
                                    int xs)
{
    const uint64_t w0 = enc[2 * t];
    const uint64_t w1 = enc[2 * t + 1];
    double v = 1.0;
    if ((w0 & 0xffffull) == 0xffffull) {
        const uint8_t *row = exps + t * n;
        for (int i = 0; i < n; ++i) {
            const uint32_t e = row[i];
            if (e) v = v * powi(x[i * xs], e);
        }
        return v;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const uint32_t ent = (uint32_t)(((s < 4 ? w0 : w1) >> (16 * (s & 3))) & 0xffffu);
        const uint32_t e = ent >> 8;
        if (e == 0) break;
        v = v * powi(x[(ent & 0xffu) * xs], e);
    }
    return v;
}

__device__ inline void store_out(const EvalArgs &A, int64_t q, int64_t pt, double y)
{
    if (A.mode == OUT_EVAL) {
        A.Y[q * A.N + pt] = y;
    } else if (A.mode == OUT_GRAD) {
        const int64_t p = q / A.n, j = q % A.n;
        A.Y[(p * A.N + pt) * A.n + j] = y;
    } else {
        const int64_t p = q / A.pairs_in_batch;
        const int64_t pi = A.pair_base + q % A.pairs_in_batch;
        const uint32_t jk = A.pair_jk[pi];
        const int64_t j = jk >> 16, k = jk & 0xffff;
        const int64_t b = (p * A.N + pt) * A.n;
        A.Y[(b + j) * A.n + k] = y;
        if (j != k) A.Y[(b + k) * A.n + j] = y;
    }
}

}  // namespace

// grid: x = blocks of 64 points, y = polynomial groups (a block loops over
// polynomials q = blockIdx.y, blockIdx.y + gridDim.y, ...).  The block's
// EV_WAVES waves share the 64 points and split each polynomial's terms
// (wave w takes terms w, w + EV_WAVES, ...); partial sums are added in wave
// order through LDS, so the result does not depend on scheduling.
// Dynamic LDS: n * 64 doubles (the block's points, variable-major).
__global__ void __launch_bounds__(EV_THREADS) k_eval_blocks(EvalArgs A, const uint64_t *enc)
{
    extern __shared__ double s_x[];
    __shared__ double s_part[EV_WAVES][kWave];
    const int lane = lane_id();
    const int w = wave_id();
    const int64_t pt0 = (int64_t)blockIdx.x * kWave;
    for (int idx = threadIdx.x; idx < A.n * kWave; idx += EV_THREADS) {
        const int i = idx / kWave, l = idx % kWave;
        const int64_t pt = pt0 + l;
        s_x[idx] = pt < A.N ? A.X[pt * A.n + i] : 0.0;
    }
    __syncthreads();
    const int64_t pt = pt0 + lane;
    const double *xl = s_x + lane;
    for (int64_t q = blockIdx.y; q < A.Q; q += gridDim.y) {
        int64_t t1 = A.rp[q + 1];
        if (t1 > A.term_limit) t1 = A.term_limit;
        double acc = 0.0;
        for (int64_t t = A.rp[q] + w; t < t1; t += EV_WAVES) acc += A.coefs[t] * term_value(enc, A.exps, A.n, t, xl, kWave);
        s_part[w][lane] = acc;
        __syncthreads();
        if (w == 0) {
            double s = s_part[0][lane];
#pragma unroll
            for (int r = 1; r < EV_WAVES; ++r) s += s_part[r][lane];
            if (pt < A.N) store_out(A, q, pt, s);
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- backward

// dX[pt, j] = sum_p gY[p, pt] * G[p, pt, j], p ascending.
__global__ void k_backward_dx(const double *G, const double *gY, int64_t P, int64_t N, int n, double *dX)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * n) return;
    const int64_t pt = idx / n;
    const int j = (int)(idx % n);
    double s = 0.0;
    for (int64_t p = 0; p < P; ++p) s += gY[p * N + pt] * G[(p * N + pt) * n + j];
    dX[idx] = s;
}

// Partial dC over one chunk of points: lanes are terms.
// grid: x = term blocks of 256, y = point chunks.  Dynamic LDS: cp * n doubles.
__global__ void __launch_bounds__(BWC_THREADS) k_backward_dc(const int64_t *rp, int64_t P, const uint8_t *exps,
                                                             int n, int64_t T, const double *X, int64_t N,
                                                             const double *gY, double *partial, int64_t nchunks,
                                                             const uint64_t *enc, int cp)
{
    extern __shared__ double s_xc[];
    const int64_t c = blockIdx.y;
    const int64_t pt0 = c * cp;
    const int np = (int)((N - pt0) < cp ? (N - pt0) : cp);
    for (int idx = threadIdx.x; idx < np * n; idx += BWC_THREADS) s_xc[idx] = X[pt0 * n + idx];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * BWC_THREADS + threadIdx.x;
    if (t >= T) return;
    int64_t lo = 0, hi = P - 1;   // polynomial of term t
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const double *g = gY + lo * N + pt0;
    double acc = 0.0;
    for (int q = 0; q < np; ++q) {
        acc += g[q] * term_value(enc, exps, n, t, s_xc + q * n, 1);
    }
    partial[c * T + t] = acc;
}

__global__ void k_backward_dc_reduce(const double *partial, int64_t T, int64_t nchunks, double *dC)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double s = partial[t];
    for (int64_t c = 1; c < nchunks; ++c) s += partial[c * T + t];
    dC[t] = s;
}

}  // namespace polyhip
