// Symbolic derivatives and sparse term-streaming evaluation.
//
//  * diff / jacobian (Section 3.3): a term with e_j > 0 becomes
//    (e - u_j, c * e_j), order preserved.  Work items of (polynomial, term
//    chunk) rank the surviving terms of each variable with wavefront ballots,
//    so the output keeps storage order without any sort.
//  * Hessian entries (jacobian(jacobian(p))): the (j, k) entry, j <= k, is
//    formed from the Jacobian with coefficient c * m, m = e_j (e_k - [j == k])
//    taken as an integer first; it is evaluated once and stored to both (j, k)
//    and (k, j).
//  * evaluation (Section 3.3, p.eval(x0)): points in lanes, terms streamed
//    wave-uniformly.  Each term is pre-encoded as the list of its factors
//    (variable indices with repetition, 16 bytes); the lane's point
//    coordinates sit in LDS, and a monomial is the left-to-right product of
//    its factors.  The waves of a workgroup share 64 points and split a
//    polynomial's terms; their partial sums are added in a fixed order.  A
//    batch whose terms all have degree <= 4 (the class the encoder records
//    on the device) is streamed by the _short kernels, which read exactly
//    that many factors per term, with no branch on the term's degree.
#include "kernels.h"

namespace polyhip {

// ------------------------------------------------- derivative formation
//
// Formed polynomial (p, g): group g of source polynomial p.  Mode 0 forms
// d/dx_g of every source polynomial (the Jacobian).  Mode 1 takes as source
// the Jacobian of f, formed with the original coefficients kept, where source
// polynomial p = (r, j) holds d/dx_j f_r; group g = k >= j forms the Hessian
// entry (j, k) with the multiplier e_j (e_k - [j = k]) of the original term,
// recovered from the Jacobian row as (e'_j + 1) e'_k, so the coefficient is
// rounded once, as in a direct second derivative.  The terms of p are cut into
// chunks of A.chunk terms; work item (p, chunk) counts,
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

// multiplier of term row `row` of source polynomial p in group g (0 = the
// term vanishes); the formed row is `row` with exponent g decremented
__device__ inline int group_mult(const FormArgs &A, const uint8_t *row, int64_t p, int64_t g)
{
    if (A.mode == 0) return row[g];
    const int jj = (int)(p % A.n);
    return g >= jj ? ((int)row[jj] + 1) * (int)row[g] : 0;
}

}  // namespace

// Rows of up to ROW_STAGE_MAX_N bytes for a block of 256 terms are staged in
// LDS by coalesced word loads, so that per-term scans of a row read LDS
// instead of issuing one divergent byte load per lane and variable.
constexpr int ROW_STAGE_MAX_N = 128;

__device__ inline void stage_rows(const uint8_t *exps, int64_t r0, int cnt, int n, uint32_t *s32)
{
    const uint8_t *src = exps + r0 * n;
    const int nb = cnt * n;
    uint8_t *s8 = reinterpret_cast<uint8_t *>(s32);
    if ((reinterpret_cast<uintptr_t>(src) & 3) == 0) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(src);
        for (int i = threadIdx.x; i < (nb >> 2); i += blockDim.x) s32[i] = w[i];
        for (int i = (nb & ~3) + threadIdx.x; i < nb; i += blockDim.x) s8[i] = src[i];
    } else {
        for (int i = threadIdx.x; i < nb; i += blockDim.x) s8[i] = src[i];
    }
}

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
    __shared__ uint32_t s_rows[JAC_THREADS * ROW_STAGE_MAX_N / 4];
    const int w = threadIdx.x >> 6;
    const bool staged = A.n <= ROW_STAGE_MAX_N;
    for (int i = threadIdx.x; i < (JAC_THREADS / kWave) * DF_MAX_GROUPS; i += JAC_THREADS) (&s_wc[0][0])[i] = 0;
    __syncthreads();
    for (int64_t c0 = t0; c0 < t1; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const int cnt = (int)(t1 - c0 < JAC_THREADS ? t1 - c0 : JAC_THREADS);
        if (staged) {
            __syncthreads();
            stage_rows(A.exps, base + c0, cnt, A.n, s_rows);
            __syncthreads();
        }
        const uint8_t *row = staged ? reinterpret_cast<const uint8_t *>(s_rows) + threadIdx.x * A.n
                                    : A.exps + (base + t) * A.n;
        for (int64_t g = 0; g < A.ngroups; ++g) {
            const int m = t < t1 ? group_mult(A, row, p, g) : 0;
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
    __shared__ uint8_t s_map[JAC_THREADS / kWave][kWave];   // survivor rank -> lane, per wave
    __shared__ int64_t s_run[DF_MAX_GROUPS];
    __shared__ uint32_t s_rows[JAC_THREADS * ROW_STAGE_MAX_N / 4];
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
    const bool staged = n <= ROW_STAGE_MAX_N;
    const bool words = (n & 3) == 0 && ((reinterpret_cast<uintptr_t>(A.exps) | reinterpret_cast<uintptr_t>(A.out_exps)) & 3) == 0;
    for (int64_t g = threadIdx.x; g < A.ngroups; g += JAC_THREADS) s_run[g] = off[cb + g * nch + chunk];
    __syncthreads();
    for (int64_t c0 = t0; c0 < t1; c0 += JAC_THREADS) {
        const int64_t t = c0 + threadIdx.x;
        const bool valid = t < t1;
        const int cnt = (int)(t1 - c0 < JAC_THREADS ? t1 - c0 : JAC_THREADS);
        if (staged) stage_rows(A.exps, base + c0, cnt, n, s_rows);
        const uint8_t *rows = staged ? reinterpret_cast<const uint8_t *>(s_rows) : A.exps + (base + c0) * n;
        if (staged) __syncthreads();
        const uint8_t *row = rows + threadIdx.x * n;
        for (int64_t g = 0; g < A.ngroups; ++g) {
            const int m = valid ? group_mult(A, row, p, g) : 0;
            const unsigned long long bal = __ballot(m > 0);
            if (lane == 0) s_wc[w][g] = __popcll(bal);
        }
        __syncthreads();
        const double c = valid ? A.coefs[base + t] : 0.0;
        for (int64_t g = 0; g < A.ngroups; ++g) {
            const int j = (int)g;
            const int m = valid ? group_mult(A, row, p, g) : 0;
            const unsigned long long bal = __ballot(m > 0);
            if (bal == 0) continue;
            // the wave's survivors take consecutive output slots from o0
            int64_t o0 = s_run[g];
            for (int q = 0; q < w; ++q) o0 += s_wc[q][g];
            const int rank = __popcll(bal & lt);
            const int nsurv = __popcll(bal);
            if (m > 0) {
                const int64_t o = o0 + rank;
                if (o < A.capacity) A.out_coefs[o] = A.keep_coefs ? c : c * (double)m;
                else set_status(A.status, A.overflow_code);
                s_map[w][rank] = (uint8_t)lane;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // their rows (exponent j decremented: it is >= 1 in a survivor) as
            // one contiguous output run, lane by lane, rows past the capacity
            // dropped
            const int64_t keep = o0 >= A.capacity ? 0 : (A.capacity - o0 < nsurv ? A.capacity - o0 : nsurv);
            if (words) {
                const uint32_t nw = (uint32_t)n >> 2;
                uint32_t *d32 = reinterpret_cast<uint32_t *>(A.out_exps + o0 * n);
                for (uint32_t d = lane; d < (uint32_t)keep * nw; d += kWave) {
                    const uint32_t r = d / nw, v = d - r * nw;
                    const uint32_t *s32 = reinterpret_cast<const uint32_t *>(rows + (w * kWave + s_map[w][r]) * n);
                    uint32_t x = s32[v];
                    if (v == (uint32_t)(j >> 2)) x -= 1u << (8 * (j & 3));
                    d32[d] = x;
                }
            } else {
                uint8_t *d8 = A.out_exps + o0 * n;
                for (uint32_t d = lane; d < (uint32_t)keep * (uint32_t)n; d += kWave) {
                    const uint32_t r = d / (uint32_t)n, v = d - r * (uint32_t)n;
                    const uint8_t *src = rows + (w * kWave + s_map[w][r]) * n;
                    d8[d] = (uint8_t)(src[v] - (v == (uint32_t)j ? 1 : 0));
                }
            }
            __builtin_amdgcn_wave_barrier();   // s_map is rewritten by the next group
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


// ---------------------------------------------------------- support encoding

// Per term: up to 8 (variable, exponent) pairs in two 64-bit words, 16 bits
// each (variable in the low byte, exponent in the high byte); unused slots are
// zero.  A term with more than eight nonzero exponents is marked 0xFFFF in the
// first slot and evaluated from its dense row.  `used` (optional, device)
// bounds the rows actually formed in a workspace of T rows.
// Rows of the block's terms: staged in LDS (n <= ROW_STAGE_MAX_N, blocks of
// at most 256 threads) or read in place.  Returns null for threads past lim.
__device__ inline const uint8_t *encode_row(const uint8_t *exps, int64_t lim, int n, uint32_t *s_rows)
{
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t t = r0 + threadIdx.x;
    const int cnt = (int)(lim - r0 < (int64_t)blockDim.x ? lim - r0 : (int64_t)blockDim.x);
    if (n <= ROW_STAGE_MAX_N) {
        stage_rows(exps, r0, cnt, n, s_rows);
        __syncthreads();
        return t < lim ? reinterpret_cast<const uint8_t *>(s_rows) + threadIdx.x * n : nullptr;
    }
    return t < lim ? exps + t * n : nullptr;
}

__global__ void __launch_bounds__(256) k_encode_support(const uint8_t *exps, int64_t T, int n, uint64_t *enc,
                                                        const int64_t *used)
{
    __shared__ uint32_t s_rows[256 * ROW_STAGE_MAX_N / 4];
    const int64_t lim = used && *used < T ? *used : T;
    if ((int64_t)blockIdx.x * blockDim.x >= lim) return;   // the whole block
    const uint8_t *row = encode_row(exps, lim, n, s_rows);
    if (!row) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// Factor-list encoding for the term-streaming evaluator: a term of total
// degree d <= EV_MAX_DEG is the list of its d variable indices with
// repetition, in variable order (x1^2 x3 -> 0, 0, 2), bytes 0..11, the rest
// of the list padded with n (an LDS row of ones); byte 12 holds d.  A term of
// higher degree has byte 12 = 0xFF and is evaluated from its dense row.
__global__ void __launch_bounds__(256) k_encode_factors(const uint8_t *exps, int64_t T, int n, uint32_t *enc,
                                                        const int64_t *used, uint32_t *maxdeg)
{
    __shared__ uint32_t s_rows[256 * ROW_STAGE_MAX_N / 4];
    const int64_t lim = used && *used < T ? *used : T;
    if ((int64_t)blockIdx.x * blockDim.x >= lim) return;   // the whole block
    const uint8_t *row = encode_row(exps, lim, n, s_rows);
    if (!row) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t w[4] = {0, 0, 0, 0};
    int d = 0;
    for (int i = 0; i < n && d <= EV_MAX_DEG; ++i) {
        for (uint32_t e = row[i]; e > 0 && d <= EV_MAX_DEG; --e) {
            if (d < EV_MAX_DEG) w[d >> 2] |= (uint32_t)i << (8 * (d & 3));
            ++d;
        }
    }
    if (d > EV_MAX_DEG) {
        w[0] = w[1] = w[2] = 0;
        w[3] = 0xFFu;
    } else {
        for (int k = d; k < EV_MAX_DEG; ++k) w[k >> 2] |= (uint32_t)n << (8 * (k & 3));
        w[3] = (uint32_t)d;
    }
    uint4 *o = reinterpret_cast<uint4 *>(enc) + t;
    *o = make_uint4(w[0], w[1], w[2], w[3]);
    if (maxdeg) {
        // the wave's largest degree, as 2 (<= 2), 3, 4 or 255 (more), by one
        // lane, and only if it raises the recorded value: the word soon holds
        // the batch's class, after which waves read it and add nothing (one
        // atomic per wave on one word would serialize on large batches)
        const uint32_t cls = w[3] <= 2u ? 2u : (w[3] <= 4u ? w[3] : 255u);
        const unsigned long long act = __ballot(1);
        const uint32_t m = __ballot(cls == 255u) ? 255u : (__ballot(cls == 4u) ? 4u : (__ballot(cls == 3u) ? 3u : 2u));
        if (lane_id() == __ffsll((long long)act) - 1 &&
            m > __hip_atomic_load(maxdeg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(maxdeg, m);
    }
}

// ------------------------------------------------------------- evaluation

namespace {

__device__ inline double powi(double x, uint32_t e)
{
    double p = x;
    for (uint32_t k = 1; k < e; ++k) p = p * x;
    return p;
}

__device__ inline void store_out(const EvalArgs &A, int64_t q, int64_t pt, double y)
{
    if (A.mode == OUT_EVAL) {
        A.Y[q * A.N + pt] = y;
    } else if (A.mode == OUT_GRAD) {
        const int64_t p = q / A.n, j = q % A.n;
        A.Y[(p * A.N + pt) * A.n + j] = y;
    } else {   // q = (p * n + j) * n + k, k >= j: staged point-contiguous for k_hess_transpose
        const int64_t k = q % A.n, j = (q / A.n) % A.n;
        if (k < j) return;
        A.Y[q * A.N + pt] = y;
    }
}

}  // namespace

namespace {

// Monomial from its dense exponent row (terms of degree > EV_MAX_DEG).
__device__ inline double monomial_dense(const uint8_t *row, int n, const double *xl)
{
    double v = 1.0;
    for (int i = 0; i < n; ++i) {
        const uint32_t e = row[i];
        if (e) v = v * powi(xl[i * kWave], e);
    }
    return v;
}

// One chunk of four factors: four variable indices packed in a word (padding
// indices point at the row of ones).  The four LDS reads are issued before
// the multiplications; the product runs left to right.
__device__ inline double chunk4(double v, uint32_t word, const double *xl)
{
    const double x0 = xl[(word & 0xffu) * kWave];
    const double x1 = xl[((word >> 8) & 0xffu) * kWave];
    const double x2 = xl[((word >> 16) & 0xffu) * kWave];
    const double x3 = xl[(word >> 24) * kWave];
    return (((v * x0) * x1) * x2) * x3;
}

// a 64-bit value that is the same on every lane, as a scalar
__device__ inline int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// value of v in lane k (k uniform)
__device__ inline double lane_f64(double v, int k)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), k);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum of c_t * m_t(x) over terms [ta, tb), in term order.  Term records
// travel in groups of 64: lane l loads the record of term g0 + l (one
// coalesced load per field), each term is read out of its lane into scalar
// registers, and the next group's loads are in flight while the current
// group is evaluated.  Only the factor words a term's degree needs are read.
__device__ inline double term_range(const EvalArgs &A, const uint32_t *enc, int64_t ta, int64_t tb,
                                    const double *xl)
{
    double acc = 0.0;
    const uint4 *ev = reinterpret_cast<const uint4 *>(enc);
    const int lane = lane_id();
    uint4 gw = make_uint4(0, 0, 0, 0);
    double gc = 0.0;
    if (ta + lane < tb) {
        gw = ev[ta + lane];
        gc = A.coefs[ta + lane];
    }
    for (int64_t g0 = ta; g0 < tb; g0 += kWave) {
        uint4 hw = make_uint4(0, 0, 0, 0);
        double hc = 0.0;
        const int64_t tn = g0 + kWave + lane;
        if (tn < tb) {
            hw = ev[tn];
            hc = A.coefs[tn];
        }
        const int cnt = (int)(tb - g0 < kWave ? tb - g0 : kWave);
        for (int k = 0; k < cnt; ++k) {
            const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)gw.w, k);
            const double c = lane_f64(gc, k);
            double v;
            if (d <= (uint32_t)EV_MAX_DEG) {
                v = 1.0;
                if (d > 0) v = chunk4(v, (uint32_t)__builtin_amdgcn_readlane((int)gw.x, k), xl);
                if (d > 4) v = chunk4(v, (uint32_t)__builtin_amdgcn_readlane((int)gw.y, k), xl);
                if (d > 8) v = chunk4(v, (uint32_t)__builtin_amdgcn_readlane((int)gw.z, k), xl);
            } else {
                v = monomial_dense(A.exps + (g0 + k) * A.n, A.n, xl);
            }
            acc += c * v;
        }
        gw = hw;
        gc = hc;
    }
    return acc;
}

// term_range for a batch whose terms all have degree <= C (C = 2, 3, 4: the
// batch's recorded largest degree class): a term is the product of the first
// C factors of its list, read with no branch on its degree.  The padding
// factors are ones, so the value is the same to the bit as term_range's.
template <int C>
__device__ inline double term_range_short(const double *__restrict__ coefs, const uint32_t *__restrict__ enc,
                                          int64_t ta, int64_t tb, const double *xl)
{
    // the range is the same on every lane: as scalars, the term records and
    // coefficients are read by scalar loads, eight terms at a time, and no
    // vector instruction moves them
    ta = uniform_i64(ta);
    tb = uniform_i64(tb);
    const uint4 *ev = reinterpret_cast<const uint4 *>(enc);
    double acc = 0.0;
    auto term = [&](uint32_t word, double c) {
        double v = 1.0 * xl[(word & 0xffu) * kWave];
        if (C > 1) v = v * xl[((word >> 8) & 0xffu) * kWave];
        if (C > 2) v = v * xl[((word >> 16) & 0xffu) * kWave];
        if (C > 3) v = v * xl[(word >> 24) * kWave];
        acc += c * v;
    };
    int64_t t = ta;
    for (; t + 8 <= tb; t += 8) {
        uint32_t wd[8];
        double cf[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            wd[k] = ev[t + k].x;
            cf[k] = coefs[t + k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) term(wd[k], cf[k]);
    }
    for (; t < tb; ++t) term(ev[t].x, coefs[t]);
    return acc;
}

// term_range_short with the factor reads the batch's degree class md (<= 4) needs
__device__ inline double term_range_md(uint32_t md, const double *__restrict__ coefs, const uint32_t *__restrict__ enc,
                                       int64_t ta, int64_t tb, const double *xl)
{
    if (md <= 2) return term_range_short<2>(coefs, enc, ta, tb, xl);
    if (md == 3) return term_range_short<3>(coefs, enc, ta, tb, xl);
    return term_range_short<4>(coefs, enc, ta, tb, xl);
}

// Which of the two forms of an evaluation kernel runs: the short one when
// the batch's degree class is recorded and at most 4, the general one
// otherwise.  Both are launched; the other returns before staging anything.
template <bool SHORT>
__device__ inline bool eval_form_runs(const EvalArgs &A, uint32_t &md)
{
    md = A.maxdeg ? *A.maxdeg : 255u;
    return SHORT == (md <= 4u);
}

}  // namespace

// grid: x = blocks of 64 points (one point per lane), y = groups of work
// units.  Unit u = (q, s): term segment s of S of polynomial q.  Each wave
// takes its own units (u = blockIdx.y * EV_WAVES + wave, then strides of
// gridDim.y * EV_WAVES), sums its segment in term order and stores it
// (S == 1) or leaves it for k_eval_reduce, which adds the segments in order;
// results therefore do not depend on scheduling.  The next unit's row
// pointers are fetched while the current unit is evaluated.  The block's
// waves share the point tile in LDS: (n + 1) * 64 doubles, variable-major,
// plus a row of ones that the factor lists use as padding.
template <bool SHORT>
__device__ inline void eval_terms_body(const EvalArgs &A, const uint32_t *__restrict__ enc,
                                       const double *__restrict__ coefs, double *partial, int64_t S)
{
    extern __shared__ double s_x[];
    uint32_t md;
    if (!eval_form_runs<SHORT>(A, md)) return;
    const int lane = lane_id();
    const int w = wave_id();
    const int64_t pt0 = (int64_t)blockIdx.x * kWave;
    const int64_t pt = pt0 + lane;
    for (int idx = threadIdx.x; idx < (A.n + 1) * kWave; idx += EV_THREADS) {
        const int i = idx / kWave, l = idx % kWave;
        const int64_t p = pt0 + l;
        s_x[idx] = i == A.n ? 1.0 : (p < A.N ? A.X[p * A.n + i] : 0.0);
    }
    __syncthreads();   // the only barrier: waves run independently from here
    const double *xl = s_x + lane;
    int vz;   // a zero the compiler treats as per-lane
    asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
    const int64_t units = A.Q * S;
    const int64_t ustride = (int64_t)gridDim.y * EV_WAVES;
    int64_t u = (int64_t)blockIdx.y * EV_WAVES + w;
    if (u >= units) return;
    int64_t r0 = A.rp[u / S + vz], r1 = A.rp[u / S + 1 + vz];
    for (; u < units; u += ustride) {
        const int64_t un = u + ustride;
        int64_t n0 = 0, n1 = 0;
        if (un < units) {
            n0 = A.rp[un / S + vz];
            n1 = A.rp[un / S + 1 + vz];
        }
        const int64_t q = u / S, sg = u % S;
        const int64_t b0 = r0;
        const int64_t b1 = r1 < A.term_limit ? r1 : A.term_limit;
        const int64_t len = b1 > b0 ? b1 - b0 : 0;
        const int64_t sa = b0 + len * sg / S, sb = b0 + len * (sg + 1) / S;
        const double acc = SHORT ? term_range_md(md, coefs, enc, sa, sb, xl) : term_range(A, enc, sa, sb, xl);
        if (pt < A.N) {
            if (S == 1) store_out(A, q, pt, acc);
            else partial[(sg * A.Q + q) * A.N + pt] = acc;
        }
        r0 = n0;
        r1 = n1;
    }
}

__global__ void __launch_bounds__(EV_THREADS) k_eval_terms(EvalArgs A, const uint32_t *enc, double *partial,
                                                           int64_t S)
{
    eval_terms_body<false>(A, enc, A.coefs, partial, S);
}

// The same for batches of degree class <= 4 (term_range_short).
__global__ void __launch_bounds__(EV_THREADS) k_eval_terms_short(EvalArgs A, const uint32_t *__restrict__ enc,
                                                                 const double *__restrict__ coefs, double *partial,
                                                                 int64_t S)
{
    eval_terms_body<true>(A, enc, coefs, partial, S);
}

// Weighted sum over polynomials of formed Jacobian entries (the reverse mode
// of eval without per-polynomial gradients):
//   out[pt][j] = sum_p gY[p][pt] * J_{p, j}(x_pt),  J_{p, j} = polynomial p * n + j.
// Unit (j, s) takes the polynomials p of segment s of S, in order, and sums
// gY * (that entry's terms summed in term order); with S > 1 the segments'
// partials [S][N][n] are added in order by k_sum_slices.
template <bool SHORT>
__device__ inline void eval_wsum_body(const EvalArgs &A, const uint32_t *__restrict__ enc,
                                      const double *__restrict__ coefs, const double *gY, int64_t P, int64_t S,
                                      double *out, double *partial)
{
    extern __shared__ double s_x[];
    uint32_t md;
    if (!eval_form_runs<SHORT>(A, md)) return;
    const int lane = lane_id();
    const int w = wave_id();
    const int n = A.n;
    const int64_t pt0 = (int64_t)blockIdx.x * kWave;
    const int64_t pt = pt0 + lane;
    for (int idx = threadIdx.x; idx < (n + 1) * kWave; idx += EV_THREADS) {
        const int i = idx / kWave, l = idx % kWave;
        const int64_t p = pt0 + l;
        s_x[idx] = i == n ? 1.0 : (p < A.N ? A.X[p * n + i] : 0.0);
    }
    __syncthreads();
    const double *xl = s_x + lane;
    const int64_t units = (int64_t)n * S;
    for (int64_t u = (int64_t)blockIdx.y * EV_WAVES + w; u < units; u += (int64_t)gridDim.y * EV_WAVES) {
        const int64_t j = u / S, sg = u % S;
        const int64_t p0 = P * sg / S, p1 = P * (sg + 1) / S;
        double acc = 0.0;
        for (int64_t p = p0; p < p1; ++p) {
            const int64_t q = p * n + j;
            const int64_t b0 = A.rp[q];
            const int64_t b1 = A.rp[q + 1] < A.term_limit ? A.rp[q + 1] : A.term_limit;
            if (b1 <= b0) continue;
            const double v = SHORT ? term_range_md(md, coefs, enc, b0, b1, xl) : term_range(A, enc, b0, b1, xl);
            const double g = pt < A.N ? gY[p * A.N + pt] : 0.0;
            acc = __builtin_fma(g, v, acc);
        }
        if (pt < A.N) {
            if (S == 1) out[pt * n + j] = acc;
            else partial[(sg * A.N + pt) * n + j] = acc;
        }
    }
}

__global__ void __launch_bounds__(EV_THREADS) k_eval_wsum(EvalArgs A, const uint32_t *enc, const double *gY,
                                                          int64_t P, int64_t S, double *out, double *partial)
{
    eval_wsum_body<false>(A, enc, A.coefs, gY, P, S, out, partial);
}

// The same for batches of degree class <= 4 (term_range_short).
__global__ void __launch_bounds__(EV_THREADS) k_eval_wsum_short(EvalArgs A, const uint32_t *__restrict__ enc,
                                                                const double *__restrict__ coefs, const double *gY,
                                                                int64_t P, int64_t S, double *out, double *partial)
{
    eval_wsum_body<true>(A, enc, coefs, gY, P, S, out, partial);
}

// H[p][pt][j][k] = stage[p][min(j,k)][max(j,k)][pt]: each Hessian entry was
// evaluated once (j <= k) into a point-contiguous staging row; both triangles
// are written from it, so H is bitwise symmetric.  Block (point tile of 32,
// row j, polynomials p = z, z + gridDim.z, ...): the rows of the tile are read
// as 256-byte runs into LDS and leave as contiguous n-element rows of H.
// Dynamic LDS: n * 33 doubles.
__global__ void __launch_bounds__(256) k_hess_transpose(const double *stage, int64_t P, int64_t N, int n, double *H)
{
    extern __shared__ double s_t[];
    constexpr int TP = 32;
    const int64_t pt0 = (int64_t)blockIdx.x * TP;
    const int j = blockIdx.y;
    for (int64_t p = blockIdx.z; p < P; p += gridDim.z) {
        for (int idx = threadIdx.x; idx < n * TP; idx += blockDim.x) {
            const int k = idx / TP, l = idx % TP;
            const int64_t pt = pt0 + l;
            const int a = j < k ? j : k, b = j < k ? k : j;
            s_t[k * (TP + 1) + l] = pt < N ? stage[((p * n + a) * n + b) * N + pt] : 0.0;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < n * TP; idx += blockDim.x) {
            const int l = idx / n, k = idx % n;
            const int64_t pt = pt0 + l;
            if (pt < N) H[((p * N + pt) * n + j) * n + k] = s_t[k * (TP + 1) + l];
        }
        __syncthreads();
    }
}

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

// Partial dC over one chunk of points: lanes are terms.  Each lane holds its
// term's factor list (k_encode_factors: up to EV_MAX_DEG variable indices,
// padded with n, the index of the one that ends every point's coordinates in
// LDS), so a term of degree <= 4 costs four LDS reads and four
// multiplications per point with no branch; longer lists take their other
// words, degrees beyond EV_MAX_DEG the exponent row.  A thread takes
// BWC_TERMS terms (BWC_THREADS apart) against one staging of the chunk.
// grid: x = term blocks of BWC_TERMS * BWC_THREADS, y = point chunks.
// Dynamic LDS: cp * (n + 1) doubles, point-major.
__global__ void __launch_bounds__(BWC_THREADS) k_backward_dc(const int64_t *rp, int64_t P, const uint8_t *exps,
                                                             int n, int64_t T, const double *X, int64_t N,
                                                             const double *gY, double *partial, int64_t nchunks,
                                                             const uint4 *fenc, int cp)
{
    extern __shared__ double s_xc[];
    const int64_t c = blockIdx.y;
    const int64_t pt0 = c * cp;
    const int np = (int)((N - pt0) < cp ? (N - pt0) : cp);
    const int ld = n + 1;
    for (int idx = threadIdx.x; idx < np * ld; idx += BWC_THREADS) {
        const int q = idx / ld, i = idx % ld;
        s_xc[idx] = i == n ? 1.0 : X[(pt0 + q) * n + i];
    }
    __syncthreads();
    for (int r = 0; r < BWC_TERMS; ++r) {
        const int64_t t = ((int64_t)blockIdx.x * BWC_TERMS + r) * BWC_THREADS + threadIdx.x;
        if (t >= T) return;
        int64_t lo = 0, hi = P - 1;   // polynomial of term t
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const double *g = gY + lo * N + pt0;
        const uint4 e = fenc[t];
        double acc = 0.0;
        if (e.w <= 4u) {
            const int i0 = (int)(e.x & 0xffu), i1 = (int)((e.x >> 8) & 0xffu);
            const int i2 = (int)((e.x >> 16) & 0xffu), i3 = (int)(e.x >> 24);
            for (int q = 0; q < np; ++q) {
                const double *xq = s_xc + q * ld;
                acc += g[q] * (((xq[i0] * xq[i1]) * xq[i2]) * xq[i3]);
            }
        } else if (e.w <= (uint32_t)EV_MAX_DEG) {
            const uint32_t wd[3] = {e.x, e.y, e.z};
            const int nw = (int)((e.w + 3) / 4);
            for (int q = 0; q < np; ++q) {
                const double *xq = s_xc + q * ld;
                double v = 1.0;
                for (int k = 0; k < nw; ++k)
                    v = (((v * xq[wd[k] & 0xffu]) * xq[(wd[k] >> 8) & 0xffu]) * xq[(wd[k] >> 16) & 0xffu]) *
                        xq[wd[k] >> 24];
                acc += g[q] * v;
            }
        } else {
            const uint8_t *row = exps + t * n;
            for (int q = 0; q < np; ++q) {
                const double *xq = s_xc + q * ld;
                double v = 1.0;
                for (int i = 0; i < n; ++i)
                    if (row[i]) v = v * powi(xq[i], row[i]);
                acc += g[q] * v;
            }
        }
        partial[c * T + t] = acc;
    }
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
