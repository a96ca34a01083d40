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

// ------------------------------------------------- derivative formation
//
// Formed polynomial (p, g): group g of source polynomial p -- variable j for
// the Jacobian, pair (j, k) of the current pair batch for the Hessian.  The
// terms of p are cut into chunks of A.chunk terms; work item (p, chunk) counts,
// for every group, how many of its terms survive (wavefront ballots), the
// counts laid out per p as [group][chunk] are scanned into output offsets, and
// the same item writes its survivors in term order.  So every formed
// polynomial keeps the source term order, with any number of workgroups per
// source polynomial.

namespace {

__device__ inline int64_t item_poly(const int64_t *item_start, int64_t P, int64_t item)
{
    int64_t lo = 0, hi = P - 1;   // last p with item_start[p] <= item
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (item_start[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// multiplier of term row `row` in group g (0 = term vanishes)
__device__ inline int group_mult(const FormArgs &A, const uint8_t *row, int64_t g, int &j, int &k)
{
    if (A.mode == 0) {
        j = (int)g;
        k = -1;
        return row[j];
    }
    const uint32_t jk = A.pair_jk[A.pair_base + g];
    j = (int)(jk >> 16);
    k = (int)(jk & 0xffff);
    return (int)row[j] * ((int)row[k] - (j == k ? 1 : 0));
}

}  // namespace

__global__ void k_item_count(const int64_t *rp, int64_t P, int64_t chunk, int64_t *items)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t T = rp[p + 1] - rp[p];
    items[p] = T <= 0 ? 1 : (T + chunk - 1) / chunk;
}

__global__ void __launch_bounds__(JAC_THREADS) k_form_count(FormArgs A)
{
    __shared__ int s_wc[JAC_THREADS / kWave][DF_MAX_GROUPS];
    const int64_t item = blockIdx.x;
    const int64_t p = item_poly(A.item_start, A.P, item);
    const int64_t nch = A.item_start[p + 1] - A.item_start[p];
    const int64_t chunk = item - A.item_start[p];
    if (chunk >= nch) return;   // grid larger than the work items (inconsistent host row_ptr)
    const int64_t base = A.rp[p];
    const int64_t T = A.rp[p + 1] - base;
    const int64_t t0 = chunk * A.chunk;
    const int64_t t1 = t0 + A.chunk < T ? t0 + A.chunk : T;
    const int w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < (JAC_THREADS / kWave) * DF_MAX_GROUPS; i += JAC_THREADS) (&s_wc[0][0])[i] = 0;
    __syncthreads();
    for (int64_t c0 = t0; c0 < t1; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const uint8_t *row = A.exps + (base + t) * A.n;
        for (int64_t g = 0; g < A.ngroups; ++g) {
            int j, k;
            const int m = t < t1 ? group_mult(A, row, g, j, k) : 0;
            const unsigned long long bal = __ballot(m > 0);
            if (lane_id() == 0) s_wc[w][g] += __popcll(bal);
        }
    }
    __syncthreads();
    const int64_t cb = A.item_start[p] * A.ngroups;
    for (int64_t g = threadIdx.x; g < A.ngroups; g += JAC_THREADS) {
        int64_t c = 0;
        for (int q = 0; q < JAC_THREADS / kWave; ++q) c += s_wc[q][g];
        A.cnt[cb + g * nch + chunk] = c;
    }
}

// out_rp[p*G + g] = offset of (p, g, chunk 0); out_rp[P*G] = total
__global__ void k_form_rowptr(FormArgs A, const int64_t *off)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t G = A.ngroups;
    if (idx > A.P * G) return;
    if (idx == A.P * G) {
        A.out_rp[idx] = off[A.item_start[A.P] * G];
        return;
    }
    const int64_t p = idx / G, g = idx % G;
    const int64_t nch = A.item_start[p + 1] - A.item_start[p];
    A.out_rp[idx] = off[A.item_start[p] * G + g * nch];
}

__global__ void __launch_bounds__(JAC_THREADS) k_form_write(FormArgs A, const int64_t *off)
{
    __shared__ int s_wc[JAC_THREADS / kWave][DF_MAX_GROUPS];
    __shared__ int64_t s_run[DF_MAX_GROUPS];
    const int64_t item = blockIdx.x;
    const int64_t p = item_poly(A.item_start, A.P, item);
    const int64_t nch = A.item_start[p + 1] - A.item_start[p];
    const int64_t chunk = item - A.item_start[p];
    if (chunk >= nch) return;   // grid larger than the work items (inconsistent host row_ptr)
    const int64_t base = A.rp[p];
    const int64_t T = A.rp[p + 1] - base;
    const int64_t t0 = chunk * A.chunk;
    const int64_t t1 = t0 + A.chunk < T ? t0 + A.chunk : T;
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t cb = A.item_start[p] * A.ngroups;
    const int n = A.n;
    for (int64_t g = threadIdx.x; g < A.ngroups; g += JAC_THREADS) s_run[g] = off[cb + g * nch + chunk];
    __syncthreads();
    for (int64_t c0 = t0; c0 < t1; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const bool valid = t < t1;
        const uint8_t *row = A.exps + (base + t) * n;
        for (int64_t g = 0; g < A.ngroups; ++g) {
            int j, k;
            const int m = valid ? group_mult(A, row, g, j, k) : 0;
            const unsigned long long bal = __ballot(m > 0);
            if (lane == 0) s_wc[w][g] = __popcll(bal);
        }
        __syncthreads();
        const double c = valid ? A.coefs[base + t] : 0.0;
        for (int64_t g = 0; g < A.ngroups; ++g) {
            int j = 0, k = -1;
            const int m = valid ? group_mult(A, row, g, j, k) : 0;
            const unsigned long long bal = __ballot(m > 0);
            if (m > 0) {
                int64_t o = s_run[g] + __popcll(bal & lt);
                for (int q = 0; q < w; ++q) o += s_wc[q][g];
                if (o < A.capacity) {
                    uint8_t *orow = A.out_exps + o * n;
                    for (int v = 0; v < n; ++v) orow[v] = row[v];
                    orow[j] = (uint8_t)(orow[j] - 1);
                    if (k >= 0) orow[k] = (uint8_t)(orow[k] - 1);
                    A.out_coefs[o] = c * (double)m;
                } else {
                    set_status(A.status, A.overflow_code);
                }
            }
        }
        __syncthreads();
        for (int64_t g = threadIdx.x; g < A.ngroups; g += JAC_THREADS) {
            int64_t sum = 0;
            for (int q = 0; q < JAC_THREADS / kWave; ++q) sum += s_wc[q][g];
            s_run[g] += sum;
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

// ---------------------------------------------------------- support encoding

// Per term: up to 8 (variable, exponent) pairs in two 64-bit words, 16 bits
// each (variable in the low byte, exponent in the high byte); unused slots are
// zero.  A term with more than eight nonzero exponents is marked 0xFFFF in the
// first slot and evaluated from its dense row.  `used` (optional, device)
// bounds the rows actually formed in a workspace of T rows.
__global__ void k_encode_support(const uint8_t *exps, int64_t T, int n, uint64_t *enc, const int64_t *used)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T || (used && t >= *used)) return;
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

namespace {

// Term data is read through the constant address space: the addresses are
// wave-uniform and the arrays are not written during the launch, so the loads
// become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) uint64_t cu64;
typedef const __attribute__((address_space(4))) double cf64;
typedef double xvec16 __attribute__((ext_vector_type(16)));

// The lane's point coordinates, held in VGPRs and read with a wave-uniform
// index (indexed register moves).
struct PointRegs16 {
    xvec16 a;
    __device__ void load(const double *x, int n)
    {
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = i < n ? x[i] : 0.0;
    }
    __device__ double get(uint32_t i) const { return a[i & 15]; }
};

struct PointRegs32 {
    xvec16 a, b;
    __device__ void load(const double *x, int n)
    {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            a[i] = i < n ? x[i] : 0.0;
            b[i] = 16 + i < n ? x[16 + i] : 0.0;
        }
    }
    __device__ double get(uint32_t i) const
    {
        double v;
        if (i < 16) v = a[i];
        else v = b[i & 15];
        return v;
    }
};

// The block's points in LDS, variable-major (n > 32).
struct PointLds {
    const double *s;
    __device__ double get(uint32_t i) const { return s[i * kWave]; }
};

template <class XS>
__device__ inline double monomial(uint64_t w0, uint64_t w1, const XS &xs, const uint8_t *row, int n)
{
    double v = 1.0;
    if ((w0 & 0xffffull) == 0xffffull) {   // more than eight factors: dense row
        for (int i = 0; i < n; ++i) {
            const uint32_t e = row[i];
            if (e) v = v * powi(xs.get((uint32_t)i), e);
        }
        return v;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const uint32_t ent = (uint32_t)(((s < 4 ? w0 : w1) >> (16 * (s & 3))) & 0xffffu);
        const uint32_t e = ent >> 8;
        if (e == 0) break;
        v = v * powi(xs.get(ent & 0xffu), e);
    }
    return v;
}

constexpr int EV_GROUP = 4;   // terms per scalar-load group

// acc += sum of c_t * m_t(x) over terms [ta, tb), in term order.  Loads of
// the next group are issued before the current group is evaluated; since
// scalar loads complete out of order, the current group is forced resident
// first (the empty asm), so that evaluating it never waits on the next loads.
template <class XS>
__device__ inline double term_range(const EvalArgs &A, const uint64_t *enc, int64_t ta, int64_t tb, const XS &xs)
{
    double acc = 0.0;
    if (ta >= tb) return acc;
    cu64 *ec = (cu64 *)enc;
    cf64 *cc = (cf64 *)A.coefs;
    uint64_t w0[EV_GROUP], w1[EV_GROUP];
    double c[EV_GROUP];
#pragma unroll
    for (int k = 0; k < EV_GROUP; ++k) {
        const int64_t t = ta + k < tb ? ta + k : tb - 1;
        w0[k] = ec[2 * t];
        w1[k] = ec[2 * t + 1];
        c[k] = cc[t];
    }
    for (int64_t t0 = ta; t0 < tb; t0 += EV_GROUP) {
#pragma unroll
        for (int k = 0; k < EV_GROUP; ++k) asm volatile("" ::"s"(w0[k]), "s"(w1[k]), "s"(c[k]) : "memory");
        uint64_t n0[EV_GROUP], n1[EV_GROUP];
        double nc[EV_GROUP];
        const int64_t tn = t0 + EV_GROUP;
#pragma unroll
        for (int k = 0; k < EV_GROUP; ++k) {
            int64_t t = tn + k < tb ? tn + k : tb - 1;
            n0[k] = ec[2 * t];
            n1[k] = ec[2 * t + 1];
            nc[k] = cc[t];
        }
#pragma unroll
        for (int k = 0; k < EV_GROUP; ++k) {
            if (t0 + k < tb) acc += c[k] * monomial(w0[k], w1[k], xs, A.exps + (t0 + k) * A.n, A.n);
        }
#pragma unroll
        for (int k = 0; k < EV_GROUP; ++k) {
            w0[k] = n0[k];
            w1[k] = n1[k];
            c[k] = nc[k];
        }
    }
    return acc;
}

}  // namespace

// grid: x = blocks of 64 points (one point per lane), y = work units
// u = (q, s) looped with stride gridDim.y: polynomial q, term segment s of S.
// The block's EV_WAVES waves cut the segment into contiguous term ranges;
// their sums are added in wave order through LDS, then over segments in
// k_eval_reduce (S > 1), so results do not depend on scheduling.
// XMODE 16 / 32: coordinates in registers (n <= XMODE); 0: in LDS
// (n * 64 doubles of dynamic LDS).
template <int XMODE>
__global__ void __launch_bounds__(EV_THREADS) k_eval_terms(EvalArgs A, const uint64_t *enc, double *partial,
                                                           int64_t S)
{
    extern __shared__ double s_x[];
    __shared__ double s_part[EV_WAVES][kWave];
    const int lane = lane_id();
    const int w = wave_id();
    const int64_t pt0 = (int64_t)blockIdx.x * kWave;
    const int64_t pt = pt0 + lane;
    PointRegs16 r16;
    PointRegs32 r32;
    PointLds xl;
    if (XMODE == 16) r16.load(A.X + (pt < A.N ? pt : 0) * A.n, A.n);
    if (XMODE == 32) r32.load(A.X + (pt < A.N ? pt : 0) * A.n, A.n);
    if (XMODE == 0) {
        for (int idx = threadIdx.x; idx < A.n * kWave; idx += EV_THREADS) {
            const int i = idx / kWave, l = idx % kWave;
            const int64_t p = pt0 + l;
            s_x[idx] = p < A.N ? A.X[p * A.n + i] : 0.0;
        }
        __syncthreads();
        xl.s = s_x + lane;
    }
    const int64_t units = A.Q * S;
    for (int64_t u = blockIdx.y; u < units; u += gridDim.y) {
        const int64_t q = u / S, sg = u % S;
        const int64_t b0 = A.rp[q];
        int64_t b1 = A.rp[q + 1];
        if (b1 > A.term_limit) b1 = A.term_limit;
        const int64_t len = b1 > b0 ? b1 - b0 : 0;
        const int64_t sa = b0 + len * sg / S, sb = b0 + len * (sg + 1) / S;
        const int64_t sl = sb - sa;
        const int64_t ta = sa + sl * w / EV_WAVES, tb = sa + sl * (w + 1) / EV_WAVES;
        double acc;
        if (XMODE == 16) acc = term_range(A, enc, ta, tb, r16);
        else if (XMODE == 32) acc = term_range(A, enc, ta, tb, r32);
        else acc = term_range(A, enc, ta, tb, xl);
        s_part[w][lane] = acc;
        __syncthreads();
        if (w == 0) {
            double sum = s_part[0][lane];
#pragma unroll
            for (int r = 1; r < EV_WAVES; ++r) sum += s_part[r][lane];
            if (pt < A.N) {
                if (S == 1) store_out(A, q, pt, sum);
                else partial[(sg * A.Q + q) * A.N + pt] = sum;
            }
        }
        __syncthreads();
    }
}

template __global__ void k_eval_terms<0>(EvalArgs, const uint64_t *, double *, int64_t);
template __global__ void k_eval_terms<16>(EvalArgs, const uint64_t *, double *, int64_t);
template __global__ void k_eval_terms<32>(EvalArgs, const uint64_t *, double *, int64_t);

// Sum of the S segment partials of (q, pt) in segment order, stored in the
// output layout of A.mode.
__global__ void k_eval_reduce(EvalArgs A, const double *partial, int64_t S)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= A.Q * A.N) return;
    const int64_t q = idx / A.N, pt = idx % A.N;
    double sum = partial[idx];
    for (int64_t s = 1; s < S; ++s) sum += partial[s * A.Q * A.N + idx];
    store_out(A, q, pt, sum);
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
