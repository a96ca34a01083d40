// times followed by simplify (Section 3.3 entrywise product; Section 6.3
// expansion-then-simplify) without writing the raw product to memory.
//
// With both operands' exponent rows packed into keys whose fields cannot
// carry (field width from max_exp_a + max_exp_b), the key of a product term
// is the integer sum Ka_i + Kb_j, and key order is the canonical order.  For
// a key range [lo, hi] and a row key Kr, the partners on the other operand
// form one contiguous interval of that operand's sorted keys, found by two
// binary searches.  So the raw product restricted to a key range can be
// generated on the fly:
//   1. pack both operands, sort each polynomial's keys (k_seg_sort);
//   2. per pair, cut the key space into buckets at quantiles of a sample of
//      raw product keys (k_mul_splitters);
//   3. per bucket (one workgroup): count its raw terms, reserve staging,
//      bisect the key range until every piece fits in LDS, generate each
//      piece's (key, i*|b|+j) pairs, sort them, and sum each run of equal
//      keys in (i, j) order -- the raw i-major order -- then write the
//      merged terms (k_mul_buckets);
//   4. scan the per-bucket counts and unpack into the CSR output.
#pragma clang fp contract(off)

#include "kernels.h"
#include "lds_sort.h"

namespace polyhip {

__global__ void k_mul_plan(const int64_t *a_rp, const int64_t *b_rp, int64_t P, int64_t *pb_count)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t raw = (a_rp[p + 1] - a_rp[p]) * (b_rp[p + 1] - b_rp[p]);
    pb_count[p] = mul_buckets_for(raw);
}

__global__ void k_mul_rowptr(const int64_t *out_off, const int64_t *pb_start, int64_t P, int64_t *out_rp,
                             int64_t nbuckets)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    int64_t b = pb_start[p];
    if (b > nbuckets) b = nbuckets;
    out_rp[p] = out_off[b];
}

// Every allocated bucket starts empty, so a bucket that the device-side plan
// does not reach (host and device row pointers disagreeing) does nothing.
__global__ void k_mul_init_buckets(MulArgs A)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.nbuckets) return;
    A.bk_pair[b] = 0;
    A.bk_lo[b] = 1;
    A.bk_hi[b] = 0;
}

// One block per pair; buckets [s_q, s_{q+1} - 1] from a sorted sample.
__global__ void __launch_bounds__(1024) k_mul_splitters(MulArgs A)
{
    __shared__ uint64_t s_smp[MUL_SAMPLE];
    const int64_t p = blockIdx.x;
    const int64_t b0 = A.pb_start[p];
    int64_t nb = A.pb_start[p + 1] - b0;
    if (b0 + nb > A.nbuckets) {
        if (threadIdx.x == 0) set_status(A.status, POLY_ERR_ARG);
        return;
    }
    if (nb <= 1) {
        if (threadIdx.x == 0 && nb == 1) {
            A.bk_pair[b0] = (int32_t)p;
            A.bk_lo[b0] = 0;
            A.bk_hi[b0] = ~0ull;
        }
        return;
    }
    const int64_t a0 = A.a_rp[p], ta = A.a_rp[p + 1] - a0;
    const int64_t bb = A.b_rp[p], tb = A.b_rp[p + 1] - bb;
    int M = 256;
    while (M < MUL_SAMPLE && (int64_t)M < 8 * nb) M <<= 1;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        const int64_t i = ((int64_t)k * ta) / M;
        const int64_t j = (int64_t)(hash32((uint32_t)k * 2654435761u ^ (uint32_t)p) % (uint32_t)tb);
        s_smp[k] = A.ka[a0 + i] + A.kb[bb + j];
    }
    __syncthreads();
    lds_sort_keys<1024>(s_smp, M);
    for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) {
        uint64_t lo = q == 0 ? 0ull : s_smp[(q * M) / nb];
        uint64_t hi = ~0ull;
        bool empty = false;
        if (q < nb - 1) {
            const uint64_t nxt = s_smp[((q + 1) * M) / nb];
            if (nxt == 0) empty = true;
            else hi = nxt - 1;
        }
        if (hi < lo) empty = true;   // equal consecutive splitters
        if (empty) {
            lo = 1;
            hi = 0;
        }
        A.bk_pair[b0 + q] = (int32_t)p;
        A.bk_lo[b0 + q] = lo;
        A.bk_hi[b0 + q] = hi;
    }
}

namespace {

// first index in s[0..m) with s[idx] >= x
__device__ inline int64_t lower_bound_u64(const uint64_t *__restrict__ s, int64_t m, uint64_t x)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (s[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index in s[0..m) with s[idx] > x
__device__ inline int64_t upper_bound_u64(const uint64_t *__restrict__ s, int64_t m, uint64_t x)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (s[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Partner interval of row key kr for product keys in [lo, hi].
__device__ inline void partner_range(const uint64_t *s, int64_t m, uint64_t kr, uint64_t lo, uint64_t hi,
                                     int64_t &l, int64_t &u)
{
    if (hi < kr) {
        l = u = 0;
        return;
    }
    l = lo <= kr ? 0 : lower_bound_u64(s, m, lo - kr);
    u = upper_bound_u64(s, m, hi - kr);
    if (u < l) u = l;
}

struct MulShared {
    uint64_t key[MUL_CAP];
    uint32_t val[MUL_CAP];
    int64_t scan[MUL_THREADS / kWave];
    uint64_t stk_lo[72];
    uint64_t stk_hi[72];
    int64_t stk_cnt[72];
    int64_t bcast;
};

struct PairView {
    const uint64_t *rows;   // row operand keys (storage order)
    int64_t nrows;
    const uint64_t *srt;    // other operand keys, sorted
    const uint32_t *perm;   // their local indices
    int64_t ns;
    bool swapped;           // rows are b's terms
    int64_t tb;             // |b_p|
    const double *ca, *cb;  // coefficient bases of a_p and b_p
};

__device__ int64_t count_range(const PairView &V, uint64_t lo, uint64_t hi, MulShared &S)
{
    int64_t c = 0;
    for (int64_t r = threadIdx.x; r < V.nrows; r += MUL_THREADS) {
        int64_t l, u;
        partner_range(V.srt, V.ns, V.rows[r], lo, hi, l, u);
        c += u - l;
    }
    return block_sum<MUL_THREADS>(c, S.scan);
}

__device__ int gather_range(const PairView &V, uint64_t lo, uint64_t hi, MulShared &S)
{
    int64_t got = 0;
    for (int64_t r0 = 0; r0 < V.nrows; r0 += MUL_THREADS) {
        const int64_t r = r0 + threadIdx.x;
        int64_t l = 0, u = 0;
        uint64_t kr = 0;
        if (r < V.nrows) {
            kr = V.rows[r];
            partner_range(V.srt, V.ns, kr, lo, hi, l, u);
        }
        int64_t tot;
        const int64_t pos = block_exclusive_scan<MUL_THREADS>(u - l, S.scan, tot);
        for (int64_t q = l; q < u; ++q) {
            const int64_t d = got + pos + (q - l);
            if (d < MUL_CAP) {
                const uint32_t o = V.perm[q];
                S.key[d] = kr + V.srt[q];
                S.val[d] = V.swapped ? (uint32_t)(o * V.tb + r) : (uint32_t)(r * V.tb + o);
            }
        }
        got += tot;
    }
    __syncthreads();
    return (int)(got < MUL_CAP ? got : MUL_CAP);
}

__device__ int64_t merge_tile(const PairView &V, const MulArgs &A, MulShared &S, int m, int64_t dst)
{
    const uint32_t tb = (uint32_t)V.tb;
    int64_t written = 0;
    for (int c0 = 0; c0 < m; c0 += MUL_THREADS) {
        const int i = c0 + threadIdx.x;
        int64_t keep = 0;
        double s = 0.0;
        uint64_t k = 0;
        if (i < m) {
            k = S.key[i];
            if (i == 0 || S.key[i - 1] != k) {
                uint32_t v = S.val[i];
                s = V.ca[v / tb] * V.cb[v % tb];
                for (int q = i + 1; q < m && S.key[q] == k; ++q) {
                    v = S.val[q];
                    s = s + V.ca[v / tb] * V.cb[v % tb];
                }
                keep = !(fabs(s) <= A.tol);
            }
        }
        int64_t tot;
        const int64_t pos = block_exclusive_scan<MUL_THREADS>(keep, S.scan, tot);
        if (keep) {
            A.st_key[dst + written + pos] = k;
            A.st_coef[dst + written + pos] = s;
        }
        written += tot;
    }
    return written;
}

}  // namespace

__global__ void __launch_bounds__(MUL_THREADS) k_mul_buckets(MulArgs A)
{
    __shared__ MulShared S;
    const int64_t b = blockIdx.x;
    const int64_t p = A.bk_pair[b];
    const uint64_t lo0 = A.bk_lo[b], hi0 = A.bk_hi[b];
    const int64_t a0 = A.a_rp[p], ta = A.a_rp[p + 1] - a0;
    const int64_t bb = A.b_rp[p], tb = A.b_rp[p + 1] - bb;
    if (lo0 > hi0 || ta == 0 || tb == 0) {
        if (threadIdx.x == 0) {
            A.bk_count[b] = 0;
            A.bk_stage_off[b] = 0;
        }
        return;
    }
    PairView V;
    V.swapped = ta > tb;
    V.tb = tb;
    V.ca = A.a_c + a0;
    V.cb = A.b_c + bb;
    if (!V.swapped) {
        V.rows = A.ka + a0;
        V.nrows = ta;
        V.srt = A.kb_s + bb;
        V.perm = A.perm_b + bb;
        V.ns = tb;
    } else {
        V.rows = A.kb + bb;
        V.nrows = tb;
        V.srt = A.ka_s + a0;
        V.perm = A.perm_a + a0;
        V.ns = ta;
    }
    const int64_t root = count_range(V, lo0, hi0, S);
    if (root == 0) {
        if (threadIdx.x == 0) {
            A.bk_count[b] = 0;
            A.bk_stage_off[b] = 0;
        }
        return;
    }
    if (threadIdx.x == 0) {
        S.bcast = (int64_t)atomicAdd(A.stage_cursor, (unsigned long long)root);
        S.stk_lo[0] = lo0;
        S.stk_hi[0] = hi0;
        S.stk_cnt[0] = root;
    }
    __syncthreads();
    const int64_t stage = S.bcast;
    if (stage + root > A.st_capacity) {
        if (threadIdx.x == 0) {
            set_status(A.status, POLY_ERR_ARG);
            A.bk_count[b] = 0;
            A.bk_stage_off[b] = 0;
        }
        return;
    }
    int64_t written = 0;
    int sp = 1;
    while (sp > 0) {
        __syncthreads();
        --sp;
        const uint64_t lo = S.stk_lo[sp], hi = S.stk_hi[sp];
        const int64_t cnt = S.stk_cnt[sp];
        __syncthreads();
        if (cnt == 0) continue;
        if (cnt <= MUL_CAP) {
            const int m = gather_range(V, lo, hi, S);
            lds_sort_kv<MUL_THREADS>(S.key, S.val, m);
            written += merge_tile(V, A, S, m, stage + written);
        } else if (lo == hi) {
            // a single product key with more raw terms than a tile: sum in
            // (i, j) order directly (rows of a in storage order, partners in
            // b's stable sorted order).
            if (threadIdx.x == 0) {
                const uint64_t *kbs = A.kb_s + bb;
                const uint32_t *pb = A.perm_b + bb;
                double s = 0.0;
                bool first = true;
                for (int64_t i = 0; i < ta; ++i) {
                    const uint64_t kai = A.ka[a0 + i];
                    if (kai > lo) continue;
                    const int64_t l = lower_bound_u64(kbs, tb, lo - kai);
                    const int64_t u = upper_bound_u64(kbs, tb, lo - kai);
                    for (int64_t q = l; q < u; ++q) {
                        const double t = V.ca[i] * V.cb[pb[q]];
                        s = first ? t : s + t;
                        first = false;
                    }
                }
                const bool keep = !(fabs(s) <= A.tol);
                if (keep) {
                    A.st_key[stage + written] = lo;
                    A.st_coef[stage + written] = s;
                }
                S.bcast = keep ? 1 : 0;
            }
            __syncthreads();
            written += S.bcast;
        } else {
            const uint64_t mid = lo + (hi - lo) / 2;
            const int64_t left = count_range(V, lo, mid, S);
            if (threadIdx.x == 0) {
                S.stk_lo[sp] = mid + 1;
                S.stk_hi[sp] = hi;
                S.stk_cnt[sp] = cnt - left;
                S.stk_lo[sp + 1] = lo;
                S.stk_hi[sp + 1] = mid;
                S.stk_cnt[sp + 1] = left;
            }
            sp += 2;
        }
    }
    if (threadIdx.x == 0) {
        A.bk_count[b] = written;
        A.bk_stage_off[b] = stage;
    }
}

}  // namespace polyhip
