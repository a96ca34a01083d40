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

__global__ void k_mul_plan(const int64_t *a_rp, const int64_t *b_rp, int64_t P, int64_t *pb_count, int64_t target)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t raw = (a_rp[p + 1] - a_rp[p]) * (b_rp[p + 1] - b_rp[p]);
    pb_count[p] = mul_buckets_for(raw, target);
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

// One block per pair; buckets [s_q, s_{q+1} - 1] at quantiles of a sample
// of raw product keys.  A splitter only has to be some key value, so the
// sample is sorted on its 24 most significant varying bits and the splitters
// are those truncated values.
constexpr int SPL_THREADS = 512;
constexpr int SPL_ITEMS = MUL_SAMPLE / SPL_THREADS;

__global__ void __launch_bounds__(SPL_THREADS) k_mul_splitters(MulArgs A)
{
    __shared__ uint64_t s_smp[MUL_SAMPLE];
    __shared__ uint32_t s_cnt[(SPL_THREADS / kWave) * 256];
    __shared__ uint32_t s_scan[SPL_THREADS / kWave];
    __shared__ uint64_t s_red[SPL_THREADS / kWave];
    const int64_t p = blockIdx.x;
    const int64_t b0 = A.pb_start[p];
    const int64_t nb = A.pb_start[p + 1] - b0;
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
    const int M = MUL_SAMPLE;
    uint64_t lmin = ~0ull, lmax = 0;
    for (int k = threadIdx.x; k < M; k += SPL_THREADS) {
        const int64_t i = ((int64_t)k * ta) / M;
        const int64_t j = (int64_t)(hash32((uint32_t)k * 2654435761u ^ (uint32_t)p) % (uint32_t)tb);
        const uint64_t key = A.ka[a0 + i] + A.kb[bb + j];
        s_smp[k] = key;
        lmin = key < lmin ? key : lmin;
        lmax = key > lmax ? key : lmax;
    }
    const uint64_t kmin = block_min_u64<SPL_THREADS>(lmin, s_red);
    const uint64_t kmax = block_max_u64<SPL_THREADS>(lmax, s_red);
    const int vbits = kmax > kmin ? 64 - __clzll((unsigned long long)(kmax - kmin)) : 0;
    const int shift = vbits > 24 ? vbits - 24 : 0;
    for (int k = threadIdx.x; k < M; k += SPL_THREADS) s_smp[k] = (s_smp[k] - kmin) >> shift;
    __syncthreads();
    lds_radix_sort_keys<SPL_THREADS, SPL_ITEMS>(s_smp, M, vbits - shift, s_cnt, s_scan);
    for (int64_t q = threadIdx.x; q < nb; q += SPL_THREADS) {
        uint64_t lo = q == 0 ? 0ull : (s_smp[(q * M) / nb] << shift) + kmin;
        uint64_t hi = ~0ull;
        bool empty = false;
        if (q < nb - 1) {
            const uint64_t nxt = (s_smp[((q + 1) * M) / nb] << shift) + kmin;
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


// Coefficients of each polynomial in its sorted key order: one block per
// polynomial, out[base + t] = c[base + perm[base + t]].
__global__ void k_mul_sorted_coefs(const int64_t *rp, const uint32_t *perm, const double *c, double *out)
{
    const int64_t base = rp[blockIdx.x], T = rp[blockIdx.x + 1] - base;
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) out[base + t] = c[base + perm[base + t]];
}

// ---------------------------------------------------------------------------
// Cursor-based bucket kernel.
//
// The partner keys (the sorted operand) sit in LDS; the partner coefficients
// in the same sorted order are read from a global copy.  Each row keeps a
// cursor (in registers) at its first
// partner whose product key is not below the current piece's lower bound;
// pieces are taken in ascending key order, so a piece [lo, hi] is exactly the
// partners between each row's cursor and the first product key above hi,
// found by galloping.  Piece boundaries come from a sorted sample of the
// bucket's raw keys (every SR-th raw term in (row, partner) order); a piece
// that still holds more than MB_CAP raw terms is bisected by key value.  Each
// piece is generated row by row with its coefficient products c_i * c_j,
// sorted by a stable LDS radix sort on its key (relative to the piece start),
// and every run of equal keys is summed left to right -- the raw (i, j)
// order.  When the row operand is b (|a| > |b|), the code (i << jbits) | j is
// appended below the key bits so the sort itself produces (key, i, j) order.
// ---------------------------------------------------------------------------

namespace {

struct MbShared {
    uint64_t key[MB_CAP];
    double val[MB_CAP];
    uint32_t cnt[(MB_THREADS / kWave) * 256];
    uint32_t scan32[MB_THREADS / kWave];
    int64_t scan[MB_THREADS / kWave];
    uint64_t red[MB_THREADS / kWave];
    uint64_t stk_lo[MB_STACK];
    uint64_t stk_hi[MB_STACK];
    int64_t bcast;
    int sp;
};

// Number of partners t >= c with s[t] + kr <= hi (galloping from c).
__device__ inline uint32_t advance_count(const uint64_t *s, uint32_t ns, uint32_t c, uint64_t kr, uint64_t hi)
{
    if (hi < kr) return 0;
    const uint64_t lim = hi - kr;   // s[t] <= lim
    if (c >= ns || s[c] > lim) return 0;
    uint32_t lo = c, step = 1;      // s[lo] <= lim
    uint32_t hi_i = c + 1;
    while (hi_i < ns && s[hi_i] <= lim) {
        lo = hi_i;
        step <<= 1;
        hi_i = c + step;
    }
    if (hi_i > ns) hi_i = ns;
    uint32_t a = lo + 1, b = hi_i;   // first t in (lo, hi_i] with s[t] > lim
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if (s[mid] <= lim) a = mid + 1;
        else b = mid;
    }
    return a - c;
}

__device__ inline int bitw(uint64_t v) { return v ? 64 - __clzll((unsigned long long)v) : 0; }

}  // namespace

__global__ void __launch_bounds__(MB_THREADS) k_mul_buckets_lds(MulArgs A)
{
    extern __shared__ uint64_t s_dyn[];
    __shared__ MbShared S;
    const int64_t b = blockIdx.x;
    const int64_t p = A.bk_pair[b];
    const uint64_t lo0 = A.bk_lo[b], hi0 = A.bk_hi[b];
    const int64_t a0 = A.a_rp[p], ta = A.a_rp[p + 1] - a0;
    const int64_t bb = A.b_rp[p], tb = A.b_rp[p + 1] - bb;
    const int tid = threadIdx.x;
    if (lo0 > hi0 || ta == 0 || tb == 0) {
        if (tid == 0) {
            A.bk_count[b] = 0;
            A.bk_stage_off[b] = 0;
        }
        return;
    }
    const bool swapped = ta > tb;
    const uint32_t nrows = (uint32_t)(swapped ? tb : ta);
    const uint32_t ns = (uint32_t)(swapped ? ta : tb);
    const uint64_t *g_rows = swapped ? A.kb + bb : A.ka + a0;
    const double *g_rcf = swapped ? A.b_c + bb : A.a_c + a0;
    const uint64_t *g_srt = swapped ? A.ka_s + a0 : A.kb_s + bb;
    const uint32_t *perm = swapped ? A.perm_a + a0 : A.perm_b + bb;
    const double *g_scf = swapped ? A.ca_s + a0 : A.cb_s + bb;   // partner coefficients, sorted order
    // term pair (i, j) coded as (i << jbits) | j; sorted below the key when swapped
    const int jbits = bitw((uint64_t)(tb - 1));
    const int ij_bits = swapped ? bitw((uint64_t)(ta - 1)) + jbits : 0;

    uint64_t *s_srt = s_dyn;   // [ns] partner keys, sorted
    for (uint32_t i = tid; i < ns; i += MB_THREADS) s_srt[i] = g_srt[i];
    __syncthreads();

    // this thread's rows [r0, r1), their keys in registers
    const uint32_t rpt = (nrows + MB_THREADS - 1) / MB_THREADS;
    const uint32_t r0 = tid * rpt < nrows ? tid * rpt : nrows;
    const uint32_t r1 = r0 + rpt < nrows ? r0 + rpt : nrows;
    uint64_t rk[MB_RPT];
    double rcf[MB_RPT];
    uint32_t cr[MB_RPT];
    uint32_t cur[MB_RPT];   // first partner of each row not yet consumed
    int64_t mine = 0;
#pragma unroll
    for (int q = 0; q < MB_RPT; ++q) {
        const uint32_t r = r0 + q;
        rk[q] = r < r1 ? g_rows[r] : 0;
        rcf[q] = r < r1 ? g_rcf[r] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < MB_RPT; ++q) {
        const uint32_t r = r0 + q;
        cr[q] = 0;
        cur[q] = 0;
        if (r < r1) {
            const uint64_t kr = rk[q];
            const uint32_t c = lo0 <= kr ? 0u : (uint32_t)lower_bound_u64(s_srt, ns, lo0 - kr);
            cur[q] = c;
            cr[q] = advance_count(s_srt, ns, c, kr, hi0);
            mine += cr[q];
        }
    }
    int64_t root;
    const int64_t ebase = block_exclusive_scan<MB_THREADS>(mine, S.scan, root);
    if (root == 0) {
        if (tid == 0) {
            A.bk_count[b] = 0;
            A.bk_stage_off[b] = 0;
        }
        return;
    }
    if (tid == 0) S.bcast = (int64_t)atomicAdd(A.stage_cursor, (unsigned long long)root);
    __syncthreads();
    const int64_t stage = S.bcast;
    if (stage + root > A.st_capacity) {
        if (tid == 0) {
            set_status(A.status, POLY_ERR_ARG);
            A.bk_count[b] = 0;
            A.bk_stage_off[b] = 0;
        }
        return;
    }

    // ---- piece boundaries from a sorted sample of the bucket's raw keys
    if (root > MB_CAP) {
        const int64_t SR = (root + MB_SAMPLE - 1) / MB_SAMPLE;          // sample rate
        const int nsamp = (int)((root + SR - 1) / SR);
        int64_t e = ebase;
        uint64_t smax = 0;
#pragma unroll
        for (int q = 0; q < MB_RPT; ++q) {
            const uint32_t r = r0 + q;
            if (r < r1) {
                const uint32_t c0 = cur[q];
                // first element of this row that falls on the sample grid
                int64_t first = ((e + SR - 1) / SR) * SR;
                for (int64_t f = first; f < e + cr[q]; f += SR) {
                    const uint64_t rel = rk[q] + s_srt[c0 + (uint32_t)(f - e)] - lo0;
                    S.key[f / SR] = rel;
                    smax = rel > smax ? rel : smax;
                }
                e += cr[q];
            }
        }
        const uint64_t sm = block_max_u64<MB_THREADS>(smax, S.red);
        lds_radix_sort_keys<MB_THREADS, MB_ITEMS>(S.key, nsamp, bitw(sm), S.cnt, S.scan32);
        int64_t step = (MB_CAP * 3 / 4) / SR;
        if (step < 1) step = 1;
        int64_t npieces = (nsamp + step - 1) / step;
        if (npieces > MB_STACK - 66) {
            npieces = MB_STACK - 66;
            step = (nsamp + npieces - 1) / npieces;
            npieces = (nsamp + step - 1) / step;
        }
        // pieces [B_q, B_{q+1} - 1] with B_0 = lo0, B_q = lo0 + sample[q*step]; pushed last-first
        if (tid == 0) {
            int sp = 0;
            uint64_t hi = hi0;
            for (int64_t q = npieces - 1; q >= 0; --q) {
                const uint64_t lo = q == 0 ? lo0 : lo0 + S.key[q * step];
                if (lo <= hi) {
                    S.stk_lo[sp] = lo;
                    S.stk_hi[sp] = hi;
                    ++sp;
                }
                if (lo == 0) break;
                hi = lo - 1;
                if (hi < lo0) break;
            }
            S.sp = sp;
        }
    } else if (tid == 0) {
        S.stk_lo[0] = lo0;
        S.stk_hi[0] = hi0;
        S.sp = 1;
    }
    __syncthreads();
    int sp = S.sp;

    int64_t written = 0;
    while (sp > 0) {
        __syncthreads();
        --sp;
        const uint64_t lo = S.stk_lo[sp], hi = S.stk_hi[sp];
        __syncthreads();
        int64_t c = 0;
#pragma unroll
        for (int q = 0; q < MB_RPT; ++q) {
            const uint32_t r = r0 + q;
            cr[q] = 0;
            if (r < r1) {
                cr[q] = advance_count(s_srt, ns, cur[q], rk[q], hi);
                c += cr[q];
            }
        }
        int64_t tot;
        int64_t pos = block_exclusive_scan<MB_THREADS>(c, S.scan, tot);
        if (tot == 0) continue;
        const int wbits = bitw(hi - lo);
        if (tot <= MB_CAP && wbits + ij_bits <= 64) {
            // ---- generate the piece in (row, partner) order with its products
            uint64_t kmax = 0;
#pragma unroll
            for (int q = 0; q < MB_RPT; ++q) {
                const uint32_t r = r0 + q;
                if (r < r1 && cr[q]) {
                    const double rc = rcf[q];
                    const uint32_t c0 = cur[q];
                    for (uint32_t t = c0; t < c0 + cr[q]; ++t, ++pos) {
                        const uint64_t rel = rk[q] + s_srt[t] - lo;
                        kmax = rel > kmax ? rel : kmax;
                        uint64_t key = rel;
                        if (swapped) key = (rel << ij_bits) | (((uint64_t)perm[t] << jbits) | r);
                        S.key[pos] = key;
                        S.val[pos] = swapped ? g_scf[t] * rc : rc * g_scf[t];
                    }
                    cur[q] = c0 + cr[q];
                }
            }
            const uint64_t relmax = block_max_u64<MB_THREADS>(kmax, S.red);
            const int m = (int)tot;
            lds_radix_sort<MB_THREADS, MB_ITEMS, double>(S.key, S.val, m, bitw(relmax) + ij_bits, S.cnt,
                                                          S.scan32);
            // ---- merge runs: thread owns sorted elements [tid*ITEMS, tid*ITEMS + ITEMS)
            const int e0 = tid * MB_ITEMS;
            double sums[MB_ITEMS];
            int64_t keepc = 0;
            uint32_t keepmask = 0;
#pragma unroll
            for (int q = 0; q < MB_ITEMS; ++q) {
                const int e = e0 + q;
                sums[q] = 0.0;
                if (e < m) {
                    const uint64_t k = S.key[e] >> ij_bits;
                    if (e == 0 || (S.key[e - 1] >> ij_bits) != k) {
                        double s = S.val[e];
                        for (int f = e + 1; f < m && (S.key[f] >> ij_bits) == k; ++f) s = s + S.val[f];
                        sums[q] = s;
                        if (!(fabs(s) <= A.tol)) {
                            keepmask |= 1u << q;
                            ++keepc;
                        }
                    }
                }
            }
            int64_t ktot;
            int64_t kpos = block_exclusive_scan<MB_THREADS>(keepc, S.scan, ktot);
#pragma unroll
            for (int q = 0; q < MB_ITEMS; ++q) {
                if (keepmask & (1u << q)) {
                    const int64_t d = stage + written + kpos;
                    A.st_key[d] = lo + (S.key[e0 + q] >> ij_bits);
                    A.st_coef[d] = sums[q];
                    ++kpos;
                }
            }
            written += ktot;
            __syncthreads();
        } else if (lo == hi) {
            // one product key with more raw terms than a tile: sum in (i, j)
            // order (a's terms in storage order, partners in b's stable order)
            if (tid == 0) {
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
                        const double t = A.a_c[a0 + i] * A.b_c[bb + pb[q]];
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
#pragma unroll
            for (int q = 0; q < MB_RPT; ++q) {
                const uint32_t r = r0 + q;
                if (r < r1) cur[q] += cr[q];
            }
            __syncthreads();
            written += S.bcast;
        } else {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (tid == 0) {
                S.stk_lo[sp] = mid + 1;
                S.stk_hi[sp] = hi;
                S.stk_lo[sp + 1] = lo;
                S.stk_hi[sp + 1] = mid;
            }
            sp += 2;
        }
    }
    if (tid == 0) {
        A.bk_count[b] = written;
        A.bk_stage_off[b] = stage;
    }
}

}  // namespace polyhip
