// C ABI entry points: argument checks, workspace layout, launch sequences.
// Declarations and their contracts are in include/polyhip.h.
#include <string.h>

#include <climits>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "kernels.h"

using namespace polyhip;

namespace polyhip {

namespace {
std::atomic<int64_t> g_mul_bucket_terms{MB_TARGET};
std::atomic<int64_t> g_seg_blocks_per_cu{2};
std::atomic<int64_t> g_eval_blocks_per_cu{16};
std::atomic<int64_t> g_mul_sort_min_raw{int64_t(1) << 20};
std::atomic<int64_t> g_simplify_wide_min{SEG_CAP + 1};
std::atomic<int64_t> g_deriv_fused_max_n{0};
std::atomic<int64_t> g_sort_digit_bits{8};
std::atomic<int64_t> g_dense_f64_rows{128};

struct TuneEntry {
    const char *name;
    std::atomic<int64_t> *value;
    int64_t lo, hi;
};
const TuneEntry kTune[] = {
    {"mul_bucket_terms", &g_mul_bucket_terms, 1024, 1 << 22},
    {"seg_blocks_per_cu", &g_seg_blocks_per_cu, 1, 16},
    {"eval_blocks_per_cu", &g_eval_blocks_per_cu, 1, 64},
    {"mul_sort_min_raw", &g_mul_sort_min_raw, 0, int64_t(1) << 62},
    {"simplify_wide_min", &g_simplify_wide_min, 1, int64_t(1) << 62},
    {"deriv_fused_max_n", &g_deriv_fused_max_n, 0, 255},
    {"sort_digit_bits", &g_sort_digit_bits, GS_MIN_BITS, GS_MAX_BITS},
    {"dense_f64_rows", &g_dense_f64_rows, 64, 128},
};
}  // namespace

// widest radix digit of the global sorts, and its number of bins
int sort_bits() { return (int)g_sort_digit_bits.load(); }
int64_t sort_bins() { return int64_t(1) << sort_bits(); }

Tunables tunables()
{
    return Tunables{g_mul_bucket_terms.load(), g_seg_blocks_per_cu.load(), g_eval_blocks_per_cu.load(),
                    g_mul_sort_min_raw.load(), g_simplify_wide_min.load(), g_deriv_fused_max_n.load(),
                    g_sort_digit_bits.load(), g_dense_f64_rows.load()};
}

}  // namespace polyhip

namespace polyhip {
poly_status dense_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t nslices,
                            size_t *ws_bytes);
poly_status dense_run(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P, const double *C,
                      int64_t N, const double *X, double *Y, poly_prec prec, int32_t nslices, void *ws,
                      size_t ws_bytes, hipStream_t stream, int64_t ys);
poly_status dense_bwd_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t nslices,
                                size_t *ws_bytes);
poly_status dense_bwd_run(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P, const double *C,
                          int64_t N, const double *X, const double *gY, double *dC, double *dX, poly_prec prec,
                          int32_t nslices, void *ws, size_t ws_bytes, hipStream_t s);
}  // namespace polyhip

namespace {

// Sequential workspace layout: the same walk sizes the query and places the
// buffers for the call, so the two can never disagree.
struct Layout {
    size_t off = kWsHeadBytes;
    size_t take(size_t bytes)
    {
        const size_t o = align_up(off, 256);
        off = o + (bytes ? bytes : 0);
        return o;
    }
    size_t total() const { return align_up(off, 256); }
};

template <class T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// the word of the workspace head beside the status word (cleared with it at
// the start of every call): the largest degree class of the terms the
// evaluation kernels stream (k_encode_factors)
uint32_t *ws_maxdeg(void *ws) { return at<uint32_t>(ws, 4); }

int device_cus()
{
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> g(mu);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

#define LAUNCH_CHECK()                                     \
    do {                                                   \
        if (hipGetLastError() != hipSuccess) return POLY_ERR_HIP; \
    } while (0)

poly_status check_csr(const poly_csr *c, bool input)
{
    if (!c) return POLY_ERR_ARG;
    if (c->nvars < 1 || c->nvars > 255) return POLY_ERR_ARG;
    if (c->npolys < 0 || c->capacity < 0) return POLY_ERR_ARG;
    if (c->max_exp < 0 || c->max_exp > 255) return POLY_ERR_ARG;
    if (!c->row_ptr) return POLY_ERR_ARG;
    if (input) {
        if (!c->row_ptr_host) return POLY_ERR_ARG;
        if (c->row_ptr_host[0] != 0) return POLY_ERR_ARG;
        for (int64_t p = 0; p < c->npolys; ++p)
            if (c->row_ptr_host[p + 1] < c->row_ptr_host[p]) return POLY_ERR_ARG;
        const int64_t T = c->row_ptr_host[c->npolys];
        if (T > c->capacity) return POLY_ERR_ARG;
        if (T > 0 && (!c->exps || !c->coefs)) return POLY_ERR_ARG;
        if (T >= (int64_t(1) << 32)) return POLY_ERR_UNSUPPORTED;
    } else {
        if (c->capacity > 0 && (!c->exps || !c->coefs)) return POLY_ERR_ARG;
    }
    return POLY_OK;
}

inline int64_t total_terms(const poly_csr *c) { return c->row_ptr_host[c->npolys]; }

inline unsigned grid1(int64_t n, int threads) { return (unsigned)std::max<int64_t>(1, ceil_div(n, threads)); }

// Clear the status word and small counters (a kernel, never a memset, so the
// sequence can be captured in a graph).
inline void clear_u64(unsigned long long *p, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid1(count, 256)), dim3(256), 0, s, p, 0ull, count);
}

// ------------------------------------------------------------ simplify plan

// Device-wide simplify (batches holding a polynomial larger than the
// simplify_wide_min tunable): keys p * radix^n + (mixed-radix monomial key)
// of key_bits bits radix-sorted with their value indices, runs merged by
// tiles.  span = radix^n, or 0 for a single polynomial (key = monomial key).
constexpr int kMaxWords = 40;   // 255 variables in words of at least 8 (radix <= 256), plus the top word

struct WidePlan {
    bool on = false;
    int key_bits = 0;
    uint32_t radix = 0;
    uint64_t span = 0;
    int64_t nbs = 0, nbm = 0;   // radix-pass tiles, merge tiles
    size_t keys0 = 0, keys1 = 0, vals0 = 0, vals1 = 0, hist = 0, hoff = 0, tmp = 0;
    size_t st_key = 0, st_ckey = 0, st_coef = 0, cnt = 0, soff = 0, ooff = 0;
    // key words (rows = true): word w covers variables [wlo[w], whi[w]),
    // least significant first; the last word starts at variable 0 and holds
    // the polynomial index above its variables when P > 1 (span = radix^whi
    // of that word then); runs are found by comparing rows past it.
    bool rows = false;
    int nwords = 0;
    int wlo[kMaxWords] = {}, whi[kMaxWords] = {}, wbits[kMaxWords] = {};
    size_t head = 0;
    // two words: the low word's keys kept in input order (low), gathered
    // into sorted order for the run heads, staged per run (st_low) and
    // decoded with the top word at unpack: no exponent row is gathered
    bool two = false;
    size_t low = 0, st_low = 0;
    // decoding: chunks of `chunk` digits (div = radix^chunk < 2^32)
    int chunk = 1;
    uint64_t div = 0, div_magic = 0;   // div_magic = floor((2^64 - 1) / div)
    uint32_t digit_magic = 0;          // floor((2^32 - 1) / radix)
};

inline int64_t max_segment(const int64_t *rph, int64_t P)
{
    int64_t m = 0;
    for (int64_t p = 0; p < P; ++p) m = std::max(m, rph[p + 1] - rph[p]);
    return m;
}

// P * radix^n: the range of the composite keys, or 0 past 2^64
inline unsigned __int128 wide_range(int64_t P, int n, uint32_t radix)
{
    unsigned __int128 r = (unsigned __int128)P;
    for (int i = 0; i < n && r <= ((unsigned __int128)1 << 64); ++i) r *= radix;
    return r <= ((unsigned __int128)1 << 64) ? r : 0;
}

// Whether the device-wide path takes a batch of P polynomials, R terms in
// all, the largest of max_seg terms, in n variables with exponents below radix.
inline bool wide_wanted(int64_t P, int64_t R, int64_t max_seg, int n, uint32_t radix)
{
    return R > 0 && R < (int64_t(1) << 32) && wide_range(P, n, radix) != 0 &&
           max_seg >= tunables().simplify_wide_min;
}

void plan_wide(WidePlan &w, Layout &L, int64_t P, int64_t R, int n, uint32_t radix)
{
    w.on = true;
    const unsigned __int128 range = wide_range(P, n, radix);
    const uint64_t kmax = (uint64_t)(range - 1);
    w.key_bits = kmax ? 64 - __builtin_clzll((unsigned long long)kmax) : 0;
    w.radix = radix;
    w.span = P > 1 ? (uint64_t)(range / (unsigned __int128)P) : 0;
    w.nbs = ceil_div(R, GS_TILE);
    w.nbm = ceil_div(R, MG_TILE);
    w.keys0 = L.take(8 * R);
    w.keys1 = L.take(8 * R);
    w.vals0 = L.take(4 * R);
    w.vals1 = L.take(4 * R);
    w.hist = L.take(8 * sort_bins() * w.nbs);
    w.hoff = L.take(8 * (sort_bins() * w.nbs + 1));
    w.tmp = L.take(8 * (ceil_div(std::max<int64_t>(sort_bins() * w.nbs, w.nbm), LB_TILE) + 2));
    w.st_key = L.take(8 * R);
    w.st_ckey = L.take(8 * R);
    w.st_coef = L.take(8 * R);
    w.cnt = L.take(8 * w.nbm);
    w.soff = L.take(8 * w.nbm);
    w.ooff = L.take(8 * (w.nbm + 1));
}

inline int bit_width_u128(unsigned __int128 v)
{
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// The cheapest cut of the composite key (p, x1..xn) into words below 2^64:
// the top word takes the polynomial index and the gt most significant
// variables, the rest go into as few words as fit, from x_n upward; the cut
// with the fewest radix passes of db-bit digits wins (ties: fewer words).
// Returns false when no cut fits kMaxWords words.
bool plan_words(WidePlan &w, int64_t P, int n, uint32_t radix, int db)
{
    const unsigned __int128 lim = (unsigned __int128)1 << 64;
    int best = INT_MAX, best_words = INT_MAX;
    for (int gt = n; gt >= 0; --gt) {
        unsigned __int128 top = P > 1 ? (unsigned __int128)P : 1;
        bool ok = true;
        for (int i = 0; i < gt && ok; ++i) {
            top *= radix;
            ok = top <= lim;
        }
        if (!ok) continue;
        int lo[kMaxWords], hi[kMaxWords], bits[kMaxWords];
        int nw = 0, passes = 0, v = n;
        while (v > gt && nw < kMaxWords - 1) {
            unsigned __int128 r = 1;
            int g = 0;
            while (v - g > gt && r * radix <= lim) {
                r *= radix;
                ++g;
            }
            lo[nw] = v - g;
            hi[nw] = v;
            bits[nw] = bit_width_u128(r - 1);
            passes += (bits[nw] + db - 1) / db;
            ++nw;
            v -= g;
        }
        if (v > gt) continue;
        lo[nw] = 0;
        hi[nw] = gt;
        bits[nw] = bit_width_u128(top - 1);
        passes += (bits[nw] + db - 1) / db;
        ++nw;
        if (passes < best || (passes == best && nw < best_words)) {
            best = passes;
            best_words = nw;
            w.nwords = nw;
            for (int k = 0; k < nw; ++k) {
                w.wlo[k] = lo[k];
                w.whi[k] = hi[k];
                w.wbits[k] = bits[k];
            }
            unsigned __int128 sp = 1;
            for (int i = 0; i < gt; ++i) sp *= radix;
            w.span = P > 1 ? (uint64_t)sp : 0;
        }
    }
    return best != INT_MAX;
}

// The device-wide simplify over key words (for composite keys past 64 bits,
// or exponents past 64 bits of bit fields).
bool plan_wide_words(WidePlan &w, Layout &L, int64_t P, int64_t R, int n, uint32_t radix)
{
    w.on = true;
    w.rows = true;
    w.radix = radix;
    if (!plan_words(w, P, n, radix, sort_bits())) return false;
    w.key_bits = 0;
    for (int k = 0; k < w.nwords; ++k) w.key_bits = std::max(w.key_bits, w.wbits[k]);
    w.nbs = ceil_div(R, GS_TILE);
    w.nbm = ceil_div(R, MG_TILE);
    w.keys0 = L.take(8 * R);
    w.keys1 = L.take(8 * R);
    w.vals0 = L.take(4 * R);
    w.vals1 = L.take(4 * R);
    w.hist = L.take(8 * sort_bins() * w.nbs);
    w.hoff = L.take(8 * (sort_bins() * w.nbs + 1));
    w.tmp = L.take(8 * (ceil_div(std::max<int64_t>(sort_bins() * w.nbs, w.nbm), LB_TILE) + 2));
    w.st_key = L.take(4 * R);   // representative term index per kept run
    w.st_ckey = L.take(8 * R);
    w.st_coef = L.take(8 * R);
    w.cnt = L.take(8 * w.nbm);
    w.soff = L.take(8 * w.nbm);
    w.ooff = L.take(8 * (w.nbm + 1));
    w.head = L.take((size_t)R);
    w.two = w.nwords == 2 && radix > 1;
    if (w.two) {
        w.low = L.take(8 * (size_t)R);
        w.st_low = L.take(8 * (size_t)R);
        w.chunk = 1;
        w.div = radix;
        while (w.div * radix <= 0xffffffffull) {
            w.div *= radix;
            ++w.chunk;
        }
        w.div_magic = ~0ull / w.div;
        w.digit_magic = 0xffffffffu / radix;
    }
    return true;
}

struct SimplifyPlan {
    size_t keys, st_key, st_coef, seg_count, order, queue;
    WidePlan wide;
    size_t total;
    bool ok = true;   // false: too many terms for the device-wide path that the exponents need
};

poly_status run_simplify(const poly_csr *in, poly_csr *out, double zero_tol, void *ws, const struct SimplifyPlan &pl,
                         hipStream_t s);
poly_status run_wide(const WidePlan &w, void *ws, int64_t P, int64_t R, int n, int bits, const double *coefs,
                     double zero_tol, poly_csr *out, hipStream_t s);
poly_status run_wide_words(const WidePlan &w, void *ws, const poly_csr *in, double zero_tol, poly_csr *out,
                           hipStream_t s);

// T terms in P polynomials (row offsets rph on the host), n variables with
// exponents below radix.  Paths: one workgroup per polynomial on bit-field
// keys; the device-wide sort on one composite key word; the device-wide sort
// over several key words.  Exponents wider than 64 bits of bit fields take
// the device-wide path whatever the sizes.
SimplifyPlan plan_simplify(int64_t P, int64_t T, const int64_t *rph, int n, uint32_t radix)
{
    Layout L;
    SimplifyPlan s;
    const int bits = bit_width_u32(radix - 1);
    const bool fields = (int64_t)n * bits <= 64;
    const bool big = T > 0 && max_segment(rph, P) >= tunables().simplify_wide_min;
    if (T > 0 && T < (int64_t(1) << 32) && (big || !fields)) {
        s.keys = s.st_key = s.st_coef = s.seg_count = s.order = s.queue = 0;
        if (fields && wide_range(P, n, radix) != 0)
            plan_wide(s.wide, L, P, T, n, radix);
        else
            s.ok = plan_wide_words(s.wide, L, P, T, n, radix);
        s.total = L.total();
        return s;
    }
    if (!fields && T > 0) {   // no path: too many terms for 32-bit element indices
        s.ok = false;
        s.keys = s.st_key = s.st_coef = s.seg_count = s.order = s.queue = 0;
        s.total = L.total();
        return s;
    }
    s.keys = L.take(8 * T);
    s.st_key = L.take(8 * T);
    s.st_coef = L.take(8 * T);
    s.seg_count = L.take(8 * P);
    s.order = L.take(8 * P);
    s.queue = L.take(8);
    s.total = L.total();
    return s;
}

// --------------------------------------------------------------- scans

inline int64_t scan_tmp_count(int64_t S) { return ceil_div(std::max<int64_t>(S, 1), LB_TILE) + 2; }

// out[0..S] = exclusive scan of in[0..S) with out[S] = total; tmp holds
// scan_tmp_count(S) entries.
void launch_scan(const int64_t *in, int64_t S, int64_t *out, int64_t *tmp, int32_t *status, hipStream_t s,
                 bool tmp_clear = false)
{
    if (S <= 2048) {
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, in, S, out);
        return;
    }
    // single pass with decoupled look-back; its state (tmp) must be zero on
    // entry: cleared here unless the caller has (tmp_clear), and left dirty
    const int64_t nt = ceil_div(S, LB_TILE);
    if (!tmp_clear) clear_u64((unsigned long long *)tmp, nt + 2, s);
    hipLaunchKernelGGL(k_scan_lookback, dim3((unsigned)nt), dim3(LB_THREADS), 0, s, in, S, out,
                       (unsigned long long *)tmp, status);
}

// ---------------------------------------------------------------- mul plan

struct MulPlan {
    size_t ka, kb, ka_s, kb_s, perm_a, perm_b, ca_s, cb_s, cnt_tmp, order_a, order_b, queues, pb_count, pb_start;
    size_t bk_pair, bk_lo, bk_hi, bk_stage_off, bk_count, out_off, cursor, st_key, st_coef;
    int64_t raw, nbuckets, target;
    bool sort_mode;         // one pair, raw product sorted globally (mulsort.hip)
    size_t gs_keys0, gs_keys1, gs_vals0, gs_vals1, gs_hist, gs_hoff, gs_tmp, gs_count, gs_soff, gs_ooff, gs_pa, gs_pb;
    int64_t gs_blocks, gs_mblocks;   // radix-pass tiles, merge tiles
    bool lds_mode;          // partner and row keys of every pair fit in LDS
    size_t lds_dyn;         // dynamic LDS bytes of the LDS bucket kernel
    size_t total;
};

poly_status plan_mul(const poly_csr *a, const poly_csr *b, MulPlan &m)
{
    const int64_t P = a->npolys;
    const int64_t Ta = total_terms(a), Tb = total_terms(b);
    int64_t raw = 0, nb = 0;
    size_t lds_max = 0;
    int64_t rows_max = 0, ns_max = 0;
    bool codes_fit = true;   // (i << bits(|b|-1)) | j fits 32 bits for every pair
    for (int64_t p = 0; p < P; ++p) {
        const int64_t ta = a->row_ptr_host[p + 1] - a->row_ptr_host[p];
        const int64_t tb = b->row_ptr_host[p + 1] - b->row_ptr_host[p];
        const int64_t r = ta * tb;
        if (r >= (int64_t(1) << 32)) return POLY_ERR_UNSUPPORTED;
        raw += r;
        const int64_t nrows = std::min(ta, tb), ns = std::max(ta, tb);
        lds_max = std::max(lds_max, mb_lds_bytes(ns, nrows));
        rows_max = std::max(rows_max, nrows);
        ns_max = std::max(ns_max, ns);
        auto bw = [](int64_t v) { return v > 0 ? 64 - __builtin_clzll((unsigned long long)v) : 0; };
        if (bw(ta - 1) + bw(tb - 1) > 32) codes_fit = false;
    }
    // one large pair: global radix sort of the raw product (raw indices are 32-bit)
    m.sort_mode = P == 1 && raw >= tunables().mul_sort_min_raw && raw < (int64_t(1) << 32) && raw > 0;
    m.lds_mode = lds_max <= MB_LDS_LIMIT && rows_max <= MB_MAX_ROWS && ns_max <= MB_MAX_PARTNERS && codes_fit;
    m.lds_dyn = std::max<size_t>(lds_max, 16);
    m.target = m.lds_mode ? tunables().mul_bucket_terms : MUL_TARGET;
    for (int64_t p = 0; p < P; ++p) {
        const int64_t ta = a->row_ptr_host[p + 1] - a->row_ptr_host[p];
        const int64_t tb = b->row_ptr_host[p + 1] - b->row_ptr_host[p];
        nb += mul_buckets_for(ta * tb, m.target);
    }
    if (nb >= (int64_t(1) << 31)) return POLY_ERR_UNSUPPORTED;
    Layout L;
    m.ka = L.take(8 * Ta);
    m.kb = L.take(8 * Tb);
    m.ka_s = L.take(8 * Ta);
    m.kb_s = L.take(8 * Tb);
    m.perm_a = L.take(4 * Ta);
    m.perm_b = L.take(4 * Tb);
    m.ca_s = L.take(8 * Ta);
    m.cb_s = L.take(8 * Tb);
    m.cnt_tmp = L.take(8 * P);
    m.order_a = L.take(8 * P);
    m.order_b = L.take(8 * P);
    m.queues = L.take(8 * 4);
    m.pb_count = L.take(8 * P);
    m.pb_start = L.take(8 * (P + 1));
    m.bk_pair = L.take(4 * nb);
    m.bk_lo = L.take(8 * nb);
    m.bk_hi = L.take(8 * nb);
    m.bk_stage_off = L.take(8 * nb);
    m.bk_count = L.take(8 * nb);
    m.out_off = L.take(8 * (nb + 1));
    m.cursor = L.take(8);
    m.st_key = L.take(8 * raw);
    m.st_coef = L.take(8 * raw);
    if (m.sort_mode) {
        m.gs_blocks = ceil_div(raw, GS_TILE);
        m.gs_keys0 = L.take(8 * raw);
        m.gs_keys1 = L.take(8 * raw);
        m.gs_vals0 = L.take(4 * raw);
        m.gs_vals1 = L.take(4 * raw);
        m.gs_hist = L.take(8 * sort_bins() * m.gs_blocks);
        m.gs_hoff = L.take(8 * (sort_bins() * m.gs_blocks + 1));
        m.gs_tmp = L.take(8 * scan_tmp_count(std::max<int64_t>(sort_bins() * m.gs_blocks, ceil_div(raw, MG_TILE))));
        m.gs_pa = L.take(16 * Ta);
        m.gs_pb = L.take(16 * Tb);
        m.gs_mblocks = ceil_div(raw, MG_TILE);
        m.gs_count = L.take(8 * m.gs_mblocks);
        m.gs_soff = L.take(8 * m.gs_mblocks);
        m.gs_ooff = L.take(8 * (m.gs_mblocks + 1));
    }
    m.raw = raw;
    m.nbuckets = nb;
    m.total = L.total();
    return POLY_OK;
}

SegArgs presort_args(const poly_csr *c, uint64_t *keys, uint64_t *sorted, uint32_t *perm, int64_t *cnt_tmp,
                     int64_t *order, unsigned long long *queue, hipStream_t s)
{
    const int64_t P = c->npolys;
    hipLaunchKernelGGL(k_order_by_size, dim3(1), dim3(1024), 0, s, c->row_ptr, P, order);
    SegArgs A;
    A.rp = c->row_ptr;
    A.keys = keys;
    A.coefs = c->coefs;
    A.order = order;
    A.P = P;
    A.queue = queue;
    A.st_key = sorted;
    A.st_coef = nullptr;
    A.st_idx = perm;
    A.seg_count = cnt_tmp;
    A.tol = 0.0;
    return A;
}

// ----------------------------------------------------------- eval helpers

struct EvalPlan {
    size_t enc;
    size_t total;
};

// Segments per polynomial for the term-streaming kernel: polynomials are cut
// into term segments only when there are too few (polynomial, point block)
// pairs to give every wave of a full machine its own unit.  Depends on sizes
// only (workspace queries call it too).
inline int64_t eval_segments(int64_t Q, int64_t N, int64_t T)
{
    if (Q <= 0 || N <= 0) return 1;
    const int64_t units = ceil_div(EV_TARGET_WAVES, ceil_div(N, kWave));
    if (Q >= units) return 1;
    int64_t S = ceil_div(units, Q);
    S = std::min<int64_t>(S, std::max<int64_t>(1, T / (Q * EV_MIN_SEGMENT)));
    return std::max<int64_t>(1, std::min<int64_t>(S, EV_MAX_SEGMENTS));
}

inline size_t eval_partial_bytes(int64_t Q, int64_t N, int64_t S) { return S > 1 ? (size_t)(8 * S * Q * N) : 0; }

void launch_eval_blocks(const EvalArgs &A, const uint32_t *enc, double *partial, int64_t S, hipStream_t s)
{
    if (A.Q <= 0 || A.N <= 0) return;
    const unsigned gx = (unsigned)ceil_div(A.N, kWave);
    // eval_blocks_per_cu workgroups per CU, each looping over work units, so
    // that the block's points are staged in LDS once for many polynomials
    const int64_t want = std::max<int64_t>(1, ((int64_t)device_cus() * tunables().eval_blocks_per_cu + gx - 1) / gx);
    const unsigned gy = (unsigned)std::min<int64_t>(std::min<int64_t>(ceil_div(A.Q * S, EV_WAVES), want), 65535);
    const size_t lds = (size_t)(A.n + 1) * kWave * sizeof(double);
    TimedLaunch tl(POLY_TIMING_TERMS, s);
    if (A.maxdeg)
        hipLaunchKernelGGL(k_eval_terms_short, dim3(gx, gy), dim3(EV_THREADS), lds, s, A, enc, A.coefs, partial, S);
    hipLaunchKernelGGL(k_eval_terms, dim3(gx, gy), dim3(EV_THREADS), lds, s, A, enc, partial, S);
    tl.done(s);
    if (S > 1) hipLaunchKernelGGL(k_eval_reduce, dim3(grid1(A.Q * A.N, 256)), dim3(256), 0, s, A, partial, S);
}

// ------------------------------------------------------- scans, formation

// Derivative formation over (polynomial, chunk) work items.  The chunk size
// depends on the term count only, so workspace queries need no device.
struct FormPlan {
    int64_t chunk = 0, W = 0, G = 0, P = 0;
    bool bounded = false;   // W is an upper bound (source sizes known only on the device)
    size_t items = 0, item_start = 0, cnt = 0, off = 0, tmp = 0;
};

inline int64_t form_chunk(int64_t T)
{
    return std::min<int64_t>(4096, std::max<int64_t>(256, align_up(ceil_div(T, 2048), 256)));
}

FormPlan plan_form_sized(int64_t P, int64_t T, int64_t W, bool bounded, int64_t G, Layout &L)
{
    FormPlan fp;
    fp.P = P;
    fp.G = G;
    fp.chunk = form_chunk(T);
    fp.W = W;
    fp.bounded = bounded;
    fp.items = L.take(8 * P);
    fp.item_start = L.take(8 * (P + 1));
    fp.cnt = L.take(8 * fp.W * G);
    fp.off = L.take(8 * (fp.W * G + 1));
    fp.tmp = L.take(8 * scan_tmp_count(std::max<int64_t>(P, fp.W * G)));
    return fp;
}

// Source polynomials with sizes known on the host.
FormPlan plan_form(const poly_csr *f, int64_t G, Layout &L)
{
    const int64_t P = f->npolys, T = total_terms(f);
    const int64_t chunk = form_chunk(T);
    int64_t W = 0;
    for (int64_t p = 0; p < P; ++p) {
        const int64_t tp = f->row_ptr_host[p + 1] - f->row_ptr_host[p];
        W += tp <= 0 ? 1 : ceil_div(tp, chunk);
    }
    return plan_form_sized(P, T, W, false, G, L);
}

// Source polynomials formed on the device: at most T_bound terms in P polys.
FormPlan plan_form_bound(int64_t P, int64_t T_bound, int64_t G, Layout &L)
{
    return plan_form_sized(P, T_bound, P + ceil_div(T_bound, form_chunk(T_bound)), true, G, L);
}

// Forms the G polynomials of every source polynomial (mode, coefficient rule,
// outputs and capacity set by the caller) with out_rp of P*G + 1 entries.
void run_form(const FormPlan &fp, FormArgs A, void *ws, hipStream_t s)
{
    int64_t *items = at<int64_t>(ws, fp.items);
    int64_t *tmp = at<int64_t>(ws, fp.tmp);
    A.P = fp.P;
    A.item_start = at<int64_t>(ws, fp.item_start);
    A.cnt = at<int64_t>(ws, fp.cnt);
    A.chunk = fp.chunk;
    A.ngroups = fp.G;
    int64_t *off = at<int64_t>(ws, fp.off);
    // with a bounded grid the counts past the real work items are never
    // written: clear them so the scan reads defined values
    if (fp.bounded) clear_u64((unsigned long long *)A.cnt, fp.W * fp.G, s);
    hipLaunchKernelGGL(k_item_count, dim3(grid1(A.P, 256)), dim3(256), 0, s, A.rp, A.P, fp.chunk, items);
    launch_scan(items, A.P, const_cast<int64_t *>(A.item_start), tmp, A.status, s);
    hipLaunchKernelGGL(k_form_count, dim3((unsigned)fp.W), dim3(JAC_THREADS), 0, s, A);
    launch_scan(A.cnt, fp.W * fp.G, off, tmp, A.status, s);
    hipLaunchKernelGGL(k_form_rowptr, dim3(grid1(A.P * fp.G + 1, 256)), dim3(256), 0, s, A, (const int64_t *)off);
    hipLaunchKernelGGL(k_form_write, dim3((unsigned)fp.W), dim3(JAC_THREADS), 0, s, A, (const int64_t *)off);
}

// --------------------------------------------------------- kernel timing

constexpr int kTimingSlots = 4;
constexpr int kTimingRing = 1024;
struct TimingState {
    std::mutex mu;
    std::atomic<bool> on{false};
    bool created = false;
    hipEvent_t ev[kTimingSlots][kTimingRing][2];
    int64_t count[kTimingSlots] = {0, 0, 0, 0};
};
TimingState g_timing;

bool lds_attr_done = false;
std::mutex lds_mu;
void ensure_lds_attrs()
{
    std::lock_guard<std::mutex> g(lds_mu);
    if (lds_attr_done) return;
    (void)hipFuncSetAttribute((const void *)k_eval_terms, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 8192);
    (void)hipFuncSetAttribute((const void *)k_eval_terms_short, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024 - 8192);
    (void)hipFuncSetAttribute((const void *)k_backward_dc, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    (void)hipFuncSetAttribute((const void *)k_backward2_dc, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    (void)hipFuncSetAttribute((const void *)k_hess_transpose, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)hipFuncSetAttribute((const void *)k_deriv_terms<DM_GRAD>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)DV_LDS_MAX);
    (void)hipFuncSetAttribute((const void *)k_deriv_terms<DM_DX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)DV_LDS_MAX);
    (void)hipFuncSetAttribute((const void *)k_deriv_terms<DM_HVP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)DV_LDS_MAX);
    (void)hipFuncSetAttribute((const void *)k_deriv_terms<DM_DIRD>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)DV_LDS_MAX);
    (void)hipFuncSetAttribute((const void *)k_mul_buckets_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)MB_LDS_LIMIT);
    (void)hipFuncSetAttribute((const void *)k_affine_normal, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)affine_lds_bytes(AN_MAX_N_LDS));
    (void)hipFuncSetAttribute((const void *)k_affine_stochastic, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)AS_LDS_BUDGET);
    lds_attr_done = true;
}

// Bound used to size formed derivative polynomials: a term with at most
// eight nonzero exponents has at most 8 first derivatives and 36 Hessian
// entries (j <= k).  Terms beyond that are still handled; if the formed
// polynomials outgrow the workspace the device reports POLY_ERR_WORKSPACE.
inline int64_t grad_terms_bound(int64_t T, int n) { return T * std::min<int64_t>(n, 8); }
inline int64_t hess_terms_bound(int64_t T, int64_t nb) { return T * std::min<int64_t>(nb, 36); }


// ------------------------------------------------ fused derivative streaming

// Launch shape of k_deriv_terms<mode> for n variables: waves per workgroup W
// and the dynamic LDS they need (point tile, direction tile, one accumulator
// block per wave), chosen for the most resident waves per CU.  Depends on
// (mode, n) only.
struct DerivShape {
    bool ok = false;
    int W = 0;
    size_t lds = 0;
    int64_t waves_per_cu = 0;
};

DerivShape deriv_shape(int mode, int n)
{
    const bool acc = mode != DM_DIRD, dir = mode == DM_HVP || mode == DM_DIRD;
    const size_t tile = (size_t)(n + 1) * kWave * 8 + (dir ? (size_t)n * kWave * 8 : 0);
    const size_t accb = acc ? (size_t)n * DV_ACC_PITCH * 8 : 0;
    DerivShape best;
    for (int W : {8, 4, 2, 1}) {
        const size_t lds = tile + (size_t)W * accb;
        if (lds > DV_LDS_MAX) continue;
        const int64_t wgs = std::min<int64_t>((int64_t)(DV_LDS_MAX / lds), 24 / W);
        const int64_t waves = W * std::max<int64_t>(wgs, 1);
        if (!best.ok || waves > best.waves_per_cu) {
            best.ok = true;
            best.W = W;
            best.lds = lds;
            best.waves_per_cu = waves;
        }
    }
    return best;
}

constexpr int64_t DV_MIN_SEGMENT = 128;   // fewest terms per segment
constexpr int64_t DV_CUS = 256;           // segment counts are planned for a full MI355X

// Term segments per work unit: enough units for two rounds of resident waves.
int64_t deriv_segments(int mode, const DerivShape &sh, int64_t P, int64_t T, int64_t N)
{
    if (P <= 0 || N <= 0 || T <= 0) return 1;
    const int64_t blocks = ceil_div(N, kWave);
    const int64_t target = DV_CUS * sh.waves_per_cu * 2;
    const bool weighted = mode == DM_DX || mode == DM_HVP;
    const int64_t per = weighted ? blocks : blocks * P;
    if (per >= target) return 1;
    int64_t S = ceil_div(target, per);
    S = std::min<int64_t>(S, std::max<int64_t>(1, T / ((weighted ? 1 : P) * DV_MIN_SEGMENT)));
    return std::max<int64_t>(1, std::min<int64_t>(S, 1024));
}

// Elements of the result of a mode: G [P][N][n], dX / ggX [N][n], ggY [P][N].
inline int64_t deriv_out_len(int mode, int64_t P, int64_t N, int n)
{
    if (mode == DM_GRAD) return P * N * n;
    if (mode == DM_DIRD) return P * N;
    return N * n;
}

struct DerivPlan {
    DerivShape sh;
    int64_t S = 1;
    size_t part = 0;
};

DerivPlan plan_deriv(int mode, int n, int64_t P, int64_t T, int64_t N, Layout &L)
{
    DerivPlan d;
    d.sh = deriv_shape(mode, n);
    d.S = deriv_segments(mode, d.sh, P, T, N);
    d.part = L.take(d.S > 1 ? (size_t)8 * d.S * deriv_out_len(mode, P, N, n) : 0);
    return d;
}

// Launches k_deriv_terms<MODE> (and the in-order sum of segment partials).
template <int MODE>
void launch_deriv(DerivArgs A, const DerivPlan &d, void *ws, hipStream_t s)
{
    if (A.N <= 0 || A.P <= 0) return;
    A.S = d.S;
    A.partial = d.S > 1 ? at<double>(ws, d.part) : nullptr;
    const unsigned gx = (unsigned)ceil_div(A.N, kWave);
    const bool weighted = MODE == DM_DX || MODE == DM_HVP;
    const int64_t units = weighted ? d.S : A.P * d.S;
    const int64_t wgs_per_cu = std::max<int64_t>(1, d.sh.waves_per_cu / d.sh.W);
    const int64_t want = std::max<int64_t>(1, ceil_div((int64_t)device_cus() * wgs_per_cu * 2, gx));
    const unsigned gy = (unsigned)std::min<int64_t>(std::min<int64_t>(ceil_div(units, d.sh.W), want), 65535);
    TimedLaunch tl(POLY_TIMING_TERMS, s);
    hipLaunchKernelGGL(k_deriv_terms<MODE>, dim3(gx, gy), dim3(d.sh.W * kWave), d.sh.lds, s, A);
    tl.done(s);
    if (d.S > 1) {
        const int64_t Lout = deriv_out_len(MODE, A.P, A.N, A.n);
        hipLaunchKernelGGL(k_sum_slices, dim3(grid1(Lout, 256)), dim3(256), 0, s, (const double *)A.partial, Lout,
                           d.S, A.out);
    }
}

DerivArgs deriv_args(const poly_csr *f, const uint64_t *enc, const double *X, int64_t N, double *out)
{
    DerivArgs A;
    memset(&A, 0, sizeof(A));
    A.rp = f->row_ptr;
    A.P = f->npolys;
    A.T = total_terms(f);
    A.exps = f->exps;
    A.coefs = f->coefs;
    A.enc = enc;
    A.n = f->nvars;
    A.X = X;
    A.N = N;
    A.out = out;
    return A;
}

struct GradPlan {
    FormPlan form;
    size_t jrp, jexps, jcoefs, jenc, part;
    int64_t cap, S;
    bool fused = false;   // k_deriv_terms straight from the source terms
    size_t enc = 0;
    DerivPlan dv;
};

// The Jacobian formed in the workspace (source order kept), encoded as
// factor lists; the partials of its evaluation: per polynomial and point
// (gradients, wsum == false) or per segment of polynomials, point and
// variable (the weighted sum over polynomials of the reverse mode).
GradPlan plan_grad_formed(const poly_csr *f, int64_t N, Layout &L, bool wsum)
{
    GradPlan g;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    g.cap = grad_terms_bound(T, n);
    g.form = plan_form(f, n, L);
    g.jrp = L.take(8 * (P * n + 1));
    g.jexps = L.take((size_t)g.cap * n);
    g.jcoefs = L.take(8 * g.cap);
    g.jenc = L.take(16 * g.cap);
    if (wsum) {
        const int64_t per = ceil_div(std::max<int64_t>(N, 1), kWave) * n;
        g.S = std::max<int64_t>(1, std::min<int64_t>({ceil_div(EV_TARGET_WAVES, per), P, 256}));
        g.part = L.take(g.S > 1 ? (size_t)8 * g.S * N * n : 0);
    } else {
        g.S = eval_segments(P * n, N, T);
        g.part = L.take(eval_partial_bytes(P * n, N, g.S));
    }
    return g;
}

GradPlan plan_grad(const poly_csr *f, int64_t N, Layout &L)
{
    GradPlan g;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    if (n <= tunables().deriv_fused_max_n && deriv_shape(DM_GRAD, n).ok) {
        g.fused = true;
        g.enc = L.take(16 * T);
        g.dv = plan_deriv(DM_GRAD, n, P, T, N, L);
        g.cap = 0;
        g.S = g.dv.S;
        return g;
    }
    return plan_grad_formed(f, N, L, false);
}

FormArgs form_args(const int64_t *rp, const uint8_t *exps, const double *coefs, int n, int mode, int keep_coefs,
                   int32_t *status, int32_t overflow_code)
{
    FormArgs A;
    memset(&A, 0, sizeof(A));
    A.rp = rp;
    A.exps = exps;
    A.coefs = coefs;
    A.n = n;
    A.mode = mode;
    A.keep_coefs = keep_coefs;
    A.status = status;
    A.overflow_code = overflow_code;
    return A;
}

// Forms the Jacobian of f in the workspace and encodes it; returns the
// evaluation arguments over it (mode and output left to the caller).
EvalArgs form_jacobian(const poly_csr *f, const double *X, int64_t N, void *ws, const GradPlan &g, hipStream_t s)
{
    const int64_t P = f->npolys;
    const int n = f->nvars;
    int32_t *status = at<int32_t>(ws, 0);
    int64_t *jrp = at<int64_t>(ws, g.jrp);
    uint8_t *jexps = at<uint8_t>(ws, g.jexps);
    double *jcoefs = at<double>(ws, g.jcoefs);
    uint32_t *jenc = at<uint32_t>(ws, g.jenc);
    FormArgs F = form_args(f->row_ptr, f->exps, f->coefs, n, 0, 0, status, (int32_t)POLY_ERR_WORKSPACE);
    F.out_rp = jrp;
    F.out_exps = jexps;
    F.out_coefs = jcoefs;
    F.capacity = g.cap;
    run_form(g.form, F, ws, s);
    hipLaunchKernelGGL(k_encode_factors, dim3(grid1(g.cap, 256)), dim3(256), 0, s, jexps, g.cap, n, jenc,
                       (const int64_t *)(jrp + P * n), ws_maxdeg(ws));
    EvalArgs A;
    memset(&A, 0, sizeof(A));
    A.maxdeg = ws_maxdeg(ws);
    A.rp = jrp;
    A.exps = jexps;
    A.coefs = jcoefs;
    A.n = n;
    A.X = X;
    A.N = N;
    A.Q = P * n;
    A.term_limit = g.cap;
    return A;
}

poly_status run_grad(const poly_csr *f, const double *X, int64_t N, double *G, void *ws, const GradPlan &g,
                     hipStream_t s)
{
    const int n = f->nvars;
    if (g.fused) {
        const int64_t T = total_terms(f);
        uint64_t *enc = at<uint64_t>(ws, g.enc);
        if (T > 0)
            hipLaunchKernelGGL(k_encode_support, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, enc,
                               (const int64_t *)nullptr);
        launch_deriv<DM_GRAD>(deriv_args(f, enc, X, N, G), g.dv, ws, s);
        LAUNCH_CHECK();
        return POLY_OK;
    }
    EvalArgs A = form_jacobian(f, X, N, ws, g, s);
    A.mode = OUT_GRAD;
    A.Y = G;
    launch_eval_blocks(A, at<uint32_t>(ws, g.jenc), at<double>(ws, g.part), g.S, s);
    LAUNCH_CHECK();
    return POLY_OK;
}

// dX[pt][j] = sum_p gY[p][pt] J_{p,j}(x_pt) from the formed Jacobian (no
// per-polynomial gradients are stored).
poly_status run_wsum(const poly_csr *f, const double *X, int64_t N, const double *gY, double *dX, void *ws,
                     const GradPlan &g, hipStream_t s)
{
    EvalArgs A = form_jacobian(f, X, N, ws, g, s);
    const int n = f->nvars;
    const unsigned gx = (unsigned)ceil_div(N, kWave);
    const int64_t units = (int64_t)n * g.S;
    const int64_t want = std::max<int64_t>(1, ((int64_t)device_cus() * tunables().eval_blocks_per_cu + gx - 1) / gx);
    const unsigned gy = (unsigned)std::min<int64_t>(std::min<int64_t>(ceil_div(units, EV_WAVES), want), 65535);
    const size_t lds = (size_t)(n + 1) * kWave * sizeof(double);
    double *part = g.S > 1 ? at<double>(ws, g.part) : nullptr;
    TimedLaunch tl(POLY_TIMING_TERMS, s);
    if (A.maxdeg)
        hipLaunchKernelGGL(k_eval_wsum_short, dim3(gx, gy), dim3(EV_THREADS), lds, s, A,
                           (const uint32_t *)at<uint32_t>(ws, g.jenc), A.coefs, gY, f->npolys, g.S, dX, part);
    hipLaunchKernelGGL(k_eval_wsum, dim3(gx, gy), dim3(EV_THREADS), lds, s, A, (const uint32_t *)at<uint32_t>(ws, g.jenc),
                       gY, f->npolys, g.S, dX, part);
    tl.done(s);
    if (g.S > 1)
        hipLaunchKernelGGL(k_sum_slices, dim3(grid1(N * n, 256)), dim3(256), 0, s, (const double *)part, N * n, g.S,
                           dX);
    LAUNCH_CHECK();
    return POLY_OK;
}

}  // namespace

namespace polyhip {

TimedLaunch::TimedLaunch(int slot, hipStream_t s)
{
    if (!g_timing.on.load()) return;
    std::lock_guard<std::mutex> g(g_timing.mu);
    if (!g_timing.on.load() || slot < 0 || slot >= kTimingSlots) return;
    const int64_t i = g_timing.count[slot]++ % kTimingRing;
    e1 = g_timing.ev[slot][i][1];
    (void)hipEventRecord(g_timing.ev[slot][i][0], s);
}

void TimedLaunch::done(hipStream_t s)
{
    if (e1) (void)hipEventRecord(e1, s);
}

}  // namespace polyhip

extern "C" {

const char *poly_strerror(int32_t status)
{
    switch (status) {
    case POLY_OK: return "ok";
    case POLY_ERR_ARG: return "invalid argument, size or shape";
    case POLY_ERR_KEY_OVERFLOW: return "packed exponent key would exceed 64 bits (no longer returned)";
    case POLY_ERR_WORKSPACE: return "workspace too small";
    case POLY_ERR_CAPACITY: return "output capacity too small";
    case POLY_ERR_EXPONENT: return "an exponent exceeds the declared max_exp";
    case POLY_ERR_UNSUPPORTED: return "shape beyond the library's limits";
    case POLY_ERR_HIP: return "HIP runtime or launch failure";
    case POLY_ERR_SCRATCH: return "work exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

poly_status poly_tune_set(const char *name, int64_t value)
{
    if (!name) return POLY_ERR_ARG;
    for (const TuneEntry &e : kTune) {
        if (strcmp(e.name, name) == 0) {
            if (value < e.lo || value > e.hi) return POLY_ERR_ARG;
            if (e.value == &g_dense_f64_rows && value != 64 && value != 128) return POLY_ERR_ARG;
            e.value->store(value);
            return POLY_OK;
        }
    }
    return POLY_ERR_ARG;
}

poly_status poly_timing_enable(int32_t enable)
{
    std::lock_guard<std::mutex> g(g_timing.mu);
    if (enable && !g_timing.created) {
        for (int sl = 0; sl < kTimingSlots; ++sl)
            for (int i = 0; i < kTimingRing; ++i)
                for (int k = 0; k < 2; ++k)
                    if (hipEventCreate(&g_timing.ev[sl][i][k]) != hipSuccess) return POLY_ERR_HIP;
        g_timing.created = true;
    }
    for (int sl = 0; sl < kTimingSlots; ++sl) g_timing.count[sl] = 0;
    g_timing.on.store(enable != 0);
    return POLY_OK;
}

poly_status poly_timing_read(int32_t slot, double *total_ms, int64_t *launches)
{
    if (slot < 0 || slot >= kTimingSlots || !total_ms || !launches) return POLY_ERR_ARG;
    std::lock_guard<std::mutex> g(g_timing.mu);
    *total_ms = 0.0;
    *launches = 0;
    if (!g_timing.created) return POLY_OK;
    const int64_t n = std::min<int64_t>(g_timing.count[slot], kTimingRing);
    for (int64_t i = 0; i < n; ++i) {
        float ms = 0.0f;
        if (hipEventSynchronize(g_timing.ev[slot][i][1]) != hipSuccess) return POLY_ERR_HIP;
        if (hipEventElapsedTime(&ms, g_timing.ev[slot][i][0], g_timing.ev[slot][i][1]) != hipSuccess)
            return POLY_ERR_HIP;
        *total_ms += ms;
    }
    *launches = n;
    return POLY_OK;
}

poly_status poly_tune_get(const char *name, int64_t *value)
{
    if (!name || !value) return POLY_ERR_ARG;
    for (const TuneEntry &e : kTune) {
        if (strcmp(e.name, name) == 0) {
            *value = e.value->load();
            return POLY_OK;
        }
    }
    return POLY_ERR_ARG;
}

poly_status poly_read_status(const void *ws, void *stream)
{
    if (!ws) return POLY_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    int32_t st = 0;
    if (hipMemcpyAsync(&st, ws, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess) return POLY_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return POLY_ERR_HIP;
    return (poly_status)st;
}

// ------------------------------------------------------------------ simplify

poly_status poly_simplify_workspace(const poly_csr *in, size_t *ws_bytes)
{
    poly_status st = check_csr(in, true);
    if (st != POLY_OK) return st;
    if (!ws_bytes) return POLY_ERR_ARG;
    const SimplifyPlan pl = plan_simplify(in->npolys, total_terms(in), in->row_ptr_host, in->nvars,
                                          (uint32_t)in->max_exp + 1);
    if (!pl.ok) return POLY_ERR_UNSUPPORTED;
    *ws_bytes = pl.total;
    return POLY_OK;
}

poly_status poly_simplify(const poly_csr *in, poly_csr *out, double zero_tol, void *ws, size_t ws_bytes,
                          void *stream)
{
    poly_status st = check_csr(in, true);
    if (st != POLY_OK) return st;
    if ((st = check_csr(out, false)) != POLY_OK) return st;
    if (out->nvars != in->nvars || out->npolys != in->npolys) return POLY_ERR_ARG;
    if (!(zero_tol >= 0.0)) return POLY_ERR_ARG;
    const int n = in->nvars;
    const int64_t P = in->npolys, T = total_terms(in);
    const SimplifyPlan pl = plan_simplify(P, T, in->row_ptr_host, n, (uint32_t)in->max_exp + 1);
    if (!pl.ok) return POLY_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < pl.total) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0) {
        clear_u64((unsigned long long *)out->row_ptr, 1, s);
        LAUNCH_CHECK();
        return POLY_OK;
    }
    return run_simplify(in, out, zero_tol, ws, pl, s);
}

namespace {

poly_status run_simplify(const poly_csr *in, poly_csr *out, double zero_tol, void *ws, const SimplifyPlan &pl,
                         hipStream_t s)
{
    const int n = in->nvars;
    const int bits = bit_width_u32((uint32_t)in->max_exp);
    const int64_t P = in->npolys, T = total_terms(in);
    int32_t *status = at<int32_t>(ws, 0);
    if (pl.wide.rows) return run_wide_words(pl.wide, ws, in, zero_tol, out, s);
    if (pl.wide.on) {
        hipLaunchKernelGGL(k_ws_keys, dim3(grid1(T, 256)), dim3(256), 0, s, in->exps, T, n, pl.wide.radix,
                           in->max_exp, in->row_ptr, P, pl.wide.span, at<uint64_t>(ws, pl.wide.keys0),
                           at<uint32_t>(ws, pl.wide.vals0), status);
        return run_wide(pl.wide, ws, P, T, n, bits, in->coefs, zero_tol, out, s);
    }
    uint64_t *keys = at<uint64_t>(ws, pl.keys);
    unsigned long long *queue = at<unsigned long long>(ws, pl.queue);
    clear_u64(queue, 1, s);
    if (T > 0)
        hipLaunchKernelGGL(k_pack, dim3(grid1(T, 256)), dim3(256), 0, s, in->exps, T, n, bits, in->max_exp, keys,
                           status);
    int64_t *order = at<int64_t>(ws, pl.order);
    hipLaunchKernelGGL(k_order_by_size, dim3(1), dim3(1024), 0, s, in->row_ptr, P, order);
    SegArgs A;
    A.rp = in->row_ptr;
    A.keys = keys;
    A.coefs = in->coefs;
    A.order = order;
    A.P = P;
    A.queue = queue;
    A.st_key = at<uint64_t>(ws, pl.st_key);
    A.st_coef = at<double>(ws, pl.st_coef);
    A.st_idx = nullptr;
    A.seg_count = at<int64_t>(ws, pl.seg_count);
    A.tol = zero_tol;
    const int64_t grid = std::min<int64_t>(P, (int64_t)device_cus() * tunables().seg_blocks_per_cu);
    hipLaunchKernelGGL(k_seg_merge, dim3((unsigned)grid), dim3(SEG_THREADS), 0, s, A);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, A.seg_count, P, out->row_ptr);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)P), dim3(256), 0, s, in->row_ptr, A.seg_count, out->row_ptr,
                       A.st_key, A.st_coef, n, bits, out->exps, out->coefs, out->capacity, status);
    LAUNCH_CHECK();
    return POLY_OK;
}

// The sorted half of the device-wide simplify: keys0 / vals0 hold the R
// composite keys and value indices (coefficient of element g: coefs[vals[g]]).
poly_status run_wide(const WidePlan &w, void *ws, int64_t P, int64_t R, int n, int bits, const double *coefs,
                     double zero_tol, poly_csr *out, hipStream_t s)
{
    int32_t *status = at<int32_t>(ws, 0);
    uint64_t *kcur = at<uint64_t>(ws, w.keys0), *knext = at<uint64_t>(ws, w.keys1);
    uint32_t *vcur = at<uint32_t>(ws, w.vals0), *vnext = at<uint32_t>(ws, w.vals1);
    int64_t *hist = at<int64_t>(ws, w.hist), *hoff = at<int64_t>(ws, w.hoff), *tmp = at<int64_t>(ws, w.tmp);
    const int64_t nb = w.nbs;
    // scan state: cleared once, then by each pass's scatter for the next scan
    const int64_t scan_state = ceil_div(std::max<int64_t>(sort_bins() * nb, w.nbm), LB_TILE) + 2;
    clear_u64((unsigned long long *)tmp, scan_state, s);
    const int passes = (w.key_bits + sort_bits() - 1) / sort_bits();
    const int db = std::max(passes ? (w.key_bits + passes - 1) / passes : GS_MIN_BITS, GS_MIN_BITS);
    const int64_t hgrid = std::min<int64_t>(ceil_div(nb, GS_HIST_THREADS / kWave), (int64_t)device_cus() * 8);
    const GsGen gen{};   // the stream is read, not generated
    auto pass = [&](auto dbc, int p) {
        constexpr int DB = decltype(dbc)::value;
        const int shift = p * DB;
        hipLaunchKernelGGL((k_gs_hist<DB, false>), dim3((unsigned)hgrid), dim3(GS_HIST_THREADS), 0, s,
                           (const uint64_t *)kcur, R, shift, nb, hist, gen);
        launch_scan(hist, ((int64_t)1 << DB) * nb, hoff, tmp, status, s, true);
        hipLaunchKernelGGL((k_gs_scatter<DB, GS_KV>), dim3((unsigned)nb), dim3(GS_SC_THREADS), 0, s,
                           (const uint64_t *)kcur, (const uint32_t *)vcur, R, shift, nb, (const int64_t *)hoff,
                           knext, vnext, 0, (unsigned long long *)tmp, scan_state, gen);
    };
    for (int p = 0; p < passes; ++p) {
        switch (db) {
        case 4: pass(std::integral_constant<int, 4>(), p); break;
        case 5: pass(std::integral_constant<int, 5>(), p); break;
        case 6: pass(std::integral_constant<int, 6>(), p); break;
        case 7: pass(std::integral_constant<int, 7>(), p); break;
        case 8: pass(std::integral_constant<int, 8>(), p); break;
        case 9: pass(std::integral_constant<int, 9>(), p); break;
        case 10: pass(std::integral_constant<int, 10>(), p); break;
        default: pass(std::integral_constant<int, 11>(), p); break;
        }
        std::swap(kcur, knext);
        std::swap(vcur, vnext);
    }
    int64_t *cnt = at<int64_t>(ws, w.cnt), *soff = at<int64_t>(ws, w.soff), *ooff = at<int64_t>(ws, w.ooff);
    uint64_t *st_key = at<uint64_t>(ws, w.st_key);
    double *st_coef = at<double>(ws, w.st_coef);
    const int64_t mgrid = std::min<int64_t>(w.nbm, (int64_t)device_cus() * MG_BLOCKS_PER_CU);
    uint64_t *st_ckey = at<uint64_t>(ws, w.st_ckey);
    hipLaunchKernelGGL(k_ws_merge, dim3((unsigned)mgrid), dim3(MG_THREADS), 0, s, (const uint64_t *)kcur,
                       (const uint32_t *)vcur, R, coefs, zero_tol, w.span, w.radix, n, bits, st_key, st_ckey,
                       st_coef, cnt, soff);
    launch_scan(cnt, w.nbm, ooff, tmp, status, s, true);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)w.nbm), dim3(256), 0, s, (const int64_t *)soff,
                       (const int64_t *)cnt, (const int64_t *)ooff, (const uint64_t *)st_key,
                       (const double *)st_coef, n, bits, out->exps, out->coefs, out->capacity, status);
    hipLaunchKernelGGL(k_ws_rowptr, dim3(grid1(P + 1, 256)), dim3(256), 0, s, P, w.span, (const uint64_t *)kcur,
                       R, (const int64_t *)soff, (const int64_t *)cnt, (const int64_t *)ooff, w.nbm,
                       (const uint64_t *)st_ckey, out->row_ptr);
    LAUNCH_CHECK();
    return POLY_OK;
}

// One stable LSD radix pass set over the `bits` low bits of kcur (digits of
// at most sort_bits() bits), vals carried; kcur / vcur end up holding the
// sorted stream.
static void radix_passes(uint64_t *&kcur, uint64_t *&knext, uint32_t *&vcur, uint32_t *&vnext, int64_t R, int64_t nb,
                  int bits, int64_t *hist, int64_t *hoff, int64_t *tmp, int64_t scan_state, int32_t *status,
                  hipStream_t s)
{
    const int passes = (bits + sort_bits() - 1) / sort_bits();
    if (passes == 0) return;
    const int db = std::max((bits + passes - 1) / passes, GS_MIN_BITS);
    const int64_t hgrid = std::min<int64_t>(ceil_div(nb, GS_HIST_THREADS / kWave), (int64_t)device_cus() * 8);
    const GsGen gen{};
    auto pass = [&](auto dbc, int p) {
        constexpr int DB = decltype(dbc)::value;
        const int shift = p * DB;
        hipLaunchKernelGGL((k_gs_hist<DB, false>), dim3((unsigned)hgrid), dim3(GS_HIST_THREADS), 0, s,
                           (const uint64_t *)kcur, R, shift, nb, hist, gen);
        launch_scan(hist, ((int64_t)1 << DB) * nb, hoff, tmp, status, s, true);
        hipLaunchKernelGGL((k_gs_scatter<DB, GS_KV>), dim3((unsigned)nb), dim3(GS_SC_THREADS), 0, s,
                           (const uint64_t *)kcur, (const uint32_t *)vcur, R, shift, nb, (const int64_t *)hoff,
                           knext, vnext, 0, (unsigned long long *)tmp, scan_state, gen);
    };
    for (int p = 0; p < passes; ++p) {
        switch (db) {
        case 4: pass(std::integral_constant<int, 4>(), p); break;
        case 5: pass(std::integral_constant<int, 5>(), p); break;
        case 6: pass(std::integral_constant<int, 6>(), p); break;
        case 7: pass(std::integral_constant<int, 7>(), p); break;
        case 8: pass(std::integral_constant<int, 8>(), p); break;
        case 9: pass(std::integral_constant<int, 9>(), p); break;
        case 10: pass(std::integral_constant<int, 10>(), p); break;
        default: pass(std::integral_constant<int, 11>(), p); break;
        }
        std::swap(kcur, knext);
        std::swap(vcur, vnext);
    }
}

// The device-wide simplify over key words: the permutation is sorted word
// by word, least significant first, each word's keys rebuilt in the current
// order before its passes; runs are then found by the top word and the
// exponent rows, summed in order, and unpacked by copying a representative
// row.
poly_status run_wide_words(const WidePlan &w, void *ws, const poly_csr *in, double zero_tol, poly_csr *out,
                           hipStream_t s)
{
    const int n = in->nvars;
    const int64_t P = in->npolys, R = total_terms(in);
    int32_t *status = at<int32_t>(ws, 0);
    uint64_t *kcur = at<uint64_t>(ws, w.keys0), *knext = at<uint64_t>(ws, w.keys1);
    uint32_t *vcur = at<uint32_t>(ws, w.vals0), *vnext = at<uint32_t>(ws, w.vals1);
    int64_t *hist = at<int64_t>(ws, w.hist), *hoff = at<int64_t>(ws, w.hoff), *tmp = at<int64_t>(ws, w.tmp);
    const int64_t nb = w.nbs;
    const int64_t scan_state = ceil_div(std::max<int64_t>(sort_bins() * nb, w.nbm), LB_TILE) + 2;
    clear_u64((unsigned long long *)tmp, scan_state, s);
    hipLaunchKernelGGL(k_ww_iota, dim3(grid1(R, 256)), dim3(256), 0, s, vcur, R);
    uint64_t *st_ckey = at<uint64_t>(ws, w.st_ckey);
    uint64_t *low_in = w.two ? at<uint64_t>(ws, w.low) : nullptr;
    // words 0 and 1 come from one pass over the rows (word 1 parked in the
    // staging buffer of the merge, free until then)
    if (w.nwords >= 2)
        hipLaunchKernelGGL(k_ww_word2, dim3(grid1(R, 256)), dim3(256), 0, s, in->exps, R, n, w.radix, in->max_exp,
                           w.wlo[0], w.whi[0], w.wlo[1], w.whi[1], (int)(w.nwords == 2 && P > 1), in->row_ptr, P,
                           kcur, low_in, st_ckey, status);
    for (int k = 0; k < w.nwords; ++k) {
        // the word's keys in input order (coalesced reads of the rows), then,
        // past the first word, gathered into the current order
        const bool top = k == w.nwords - 1;
        if (k == 0 && w.nwords == 1)
            hipLaunchKernelGGL(k_ww_word, dim3(grid1(R, 256)), dim3(256), 0, s, in->exps, R, n, w.radix,
                               in->max_exp, w.wlo[0], w.whi[0], (int)(P > 1), in->row_ptr, P, kcur, status);
        if (k >= 2)
            hipLaunchKernelGGL(k_ww_word, dim3(grid1(R, 256)), dim3(256), 0, s, in->exps, R, n, w.radix,
                               in->max_exp, w.wlo[k], w.whi[k], (int)(top && P > 1), in->row_ptr, P, knext, status);
        if (k > 0)
            hipLaunchKernelGGL(k_ww_gather, dim3(grid1(R, 256)), dim3(256), 0, s,
                               (const uint64_t *)(k == 1 ? st_ckey : knext), (const uint32_t *)vcur, R, kcur);
        radix_passes(kcur, knext, vcur, vnext, R, nb, w.wbits[k], hist, hoff, tmp, scan_state, status, s);
    }
    uint8_t *head = at<uint8_t>(ws, w.head);
    uint64_t *low = nullptr, *st_low = nullptr;
    if (w.two) {   // the low word in sorted order (knext is free after the passes)
        low = knext;
        st_low = at<uint64_t>(ws, w.st_low);
        hipLaunchKernelGGL(k_ww_gather, dim3(grid1(R, 256)), dim3(256), 0, s, (const uint64_t *)low_in,
                           (const uint32_t *)vcur, R, low);
        hipLaunchKernelGGL(k_ww_heads2, dim3(grid1(R, 256)), dim3(256), 0, s, (const uint64_t *)kcur,
                           (const uint64_t *)low, R, head);
    } else {
        hipLaunchKernelGGL(k_ww_heads, dim3(grid1(R, 256)), dim3(256), 0, s, (const uint64_t *)kcur,
                           (const uint32_t *)vcur, R, in->exps, n, w.whi[w.nwords - 1], head);
    }
    int64_t *cnt = at<int64_t>(ws, w.cnt), *soff = at<int64_t>(ws, w.soff), *ooff = at<int64_t>(ws, w.ooff);
    uint32_t *st_idx = at<uint32_t>(ws, w.st_key);
    double *st_coef = at<double>(ws, w.st_coef);
    const int64_t mgrid = std::min<int64_t>(w.nbm, (int64_t)device_cus() * MG_BLOCKS_PER_CU);
    hipLaunchKernelGGL(k_ww_merge, dim3((unsigned)mgrid), dim3(MG_THREADS), 0, s, (const uint64_t *)kcur,
                       (const uint32_t *)vcur, (const uint8_t *)head, R, in->coefs, zero_tol, st_idx, st_ckey,
                       st_coef, cnt, soff, (const uint64_t *)low, st_low);
    launch_scan(cnt, w.nbm, ooff, tmp, status, s, true);
    if (w.two)
        hipLaunchKernelGGL(k_ww_compact2, dim3((unsigned)w.nbm, MG_TILE / 256), dim3(256), (size_t)256 * n, s,
                           (const int64_t *)soff, (const int64_t *)cnt, (const int64_t *)ooff,
                           (const uint64_t *)st_ckey, (const uint64_t *)st_low, (const double *)st_coef, n,
                           w.whi[1], (uint64_t)w.radix, w.chunk, w.div, w.div_magic, w.digit_magic, out->exps,
                           out->coefs, out->capacity, status);
    else
        hipLaunchKernelGGL(k_ww_compact, dim3((unsigned)w.nbm, MG_TILE / 256), dim3(256), 0, s,
                           (const int64_t *)soff, (const int64_t *)cnt, (const int64_t *)ooff,
                           (const uint32_t *)st_idx, (const double *)st_coef, in->exps, n, out->exps, out->coefs,
                           out->capacity, status);
    hipLaunchKernelGGL(k_ws_rowptr, dim3(grid1(P + 1, 256)), dim3(256), 0, s, P, w.span, (const uint64_t *)kcur,
                       R, (const int64_t *)soff, (const int64_t *)cnt, (const int64_t *)ooff, w.nbm,
                       (const uint64_t *)st_ckey, out->row_ptr);
    LAUNCH_CHECK();
    return POLY_OK;
}

}  // namespace

// ----------------------------------------------------------------------- mul

namespace {

// times of pairs whose exponent sums do not fit 64 bits of bit fields: the
// raw products are written out as exponent rows in the order of the
// definition and simplified by the device-wide path over key words.
struct RowsMulPlan {
    SimplifyPlan sp;
    std::vector<int64_t> rph;
    size_t re = 0, rc = 0, rrp = 0, sizes = 0, tmp = 0, total = 0;
    int64_t raw = 0;
};

static bool mul_needs_rows(const poly_csr *a, const poly_csr *b)
{
    return (int64_t)a->nvars * bit_width_u32((uint32_t)(a->max_exp + b->max_exp)) > 64;
}

static poly_status plan_mul_rows(const poly_csr *a, const poly_csr *b, RowsMulPlan &m)
{
    const int64_t P = a->npolys;
    const int n = a->nvars;
    m.rph.assign(P + 1, 0);
    for (int64_t p = 0; p < P; ++p)
        m.rph[p + 1] = m.rph[p] + (a->row_ptr_host[p + 1] - a->row_ptr_host[p]) *
                                      (b->row_ptr_host[p + 1] - b->row_ptr_host[p]);
    m.raw = m.rph[P];
    if (m.raw >= (int64_t(1) << 32)) return POLY_ERR_UNSUPPORTED;
    m.sp = plan_simplify(P, m.raw, m.rph.data(), n, (uint32_t)(a->max_exp + b->max_exp) + 1);
    if (!m.sp.ok) return POLY_ERR_UNSUPPORTED;
    Layout L;
    L.off = m.sp.total;
    m.re = L.take((size_t)m.raw * n);
    m.rc = L.take(8 * (size_t)m.raw);
    m.rrp = L.take(8 * (size_t)(P + 1));
    m.sizes = L.take(8 * (size_t)std::max<int64_t>(P, 1));
    m.tmp = L.take(8 * (size_t)scan_tmp_count(P));
    m.total = L.total();
    return POLY_OK;
}

static poly_status run_mul_rows(const poly_csr *a, const poly_csr *b, poly_csr *out, double zero_tol, void *ws,
                         RowsMulPlan &m, hipStream_t s)
{
    const int64_t P = a->npolys;
    const int n = a->nvars;
    int32_t *status = at<int32_t>(ws, 0);
    int64_t *sizes = at<int64_t>(ws, m.sizes), *rrp = at<int64_t>(ws, m.rrp);
    uint8_t *re = at<uint8_t>(ws, m.re);
    double *rc = at<double>(ws, m.rc);
    hipLaunchKernelGGL(k_mul_raw_sizes, dim3(grid1(P, 256)), dim3(256), 0, s, a->row_ptr, b->row_ptr, P, sizes);
    launch_scan(sizes, P, rrp, at<int64_t>(ws, m.tmp), status, s);
    if (m.raw > 0)
        hipLaunchKernelGGL(k_mul_expand_rows, dim3(grid1(m.raw, 256)), dim3(256), 0, s, a->row_ptr, a->exps,
                           a->coefs, a->max_exp, b->row_ptr, b->exps, b->coefs, b->max_exp, P, n,
                           (const int64_t *)rrp, m.raw, re, rc, status);
    poly_csr R;
    R.nvars = n;
    R.max_exp = a->max_exp + b->max_exp;
    R.npolys = P;
    R.capacity = m.raw;
    R.row_ptr_host = m.rph.data();
    R.row_ptr = rrp;
    R.exps = re;
    R.coefs = rc;
    return run_simplify(&R, out, zero_tol, ws, m.sp, s);
}

}  // namespace

poly_status poly_mul_workspace(const poly_csr *a, const poly_csr *b, size_t *ws_bytes, int64_t *raw_terms)
{
    poly_status st = check_csr(a, true);
    if (st != POLY_OK) return st;
    if ((st = check_csr(b, true)) != POLY_OK) return st;
    if (a->nvars != b->nvars || a->npolys != b->npolys) return POLY_ERR_ARG;
    if (mul_needs_rows(a, b)) {
        if (a->max_exp + b->max_exp > 255) return POLY_ERR_UNSUPPORTED;
        RowsMulPlan r;
        if ((st = plan_mul_rows(a, b, r)) != POLY_OK) return st;
        if (ws_bytes) *ws_bytes = r.total;
        if (raw_terms) *raw_terms = r.raw;
        return POLY_OK;
    }
    MulPlan m;
    if ((st = plan_mul(a, b, m)) != POLY_OK) return st;
    if (ws_bytes) *ws_bytes = m.total;
    if (raw_terms) *raw_terms = m.raw;
    return POLY_OK;
}

poly_status poly_mul(const poly_csr *a, const poly_csr *b, poly_csr *out, double zero_tol, void *ws,
                     size_t ws_bytes, void *stream)
{
    poly_status st = check_csr(a, true);
    if (st != POLY_OK) return st;
    if ((st = check_csr(b, true)) != POLY_OK) return st;
    if ((st = check_csr(out, false)) != POLY_OK) return st;
    if (a->nvars != b->nvars || a->npolys != b->npolys) return POLY_ERR_ARG;
    if (out->nvars != a->nvars || out->npolys != a->npolys) return POLY_ERR_ARG;
    if (!(zero_tol >= 0.0)) return POLY_ERR_ARG;
    if (a->max_exp + b->max_exp > 255) return POLY_ERR_UNSUPPORTED;
    const int n = a->nvars;
    const int bits = bit_width_u32((uint32_t)(a->max_exp + b->max_exp));
    if (mul_needs_rows(a, b)) {
        RowsMulPlan r;
        if ((st = plan_mul_rows(a, b, r)) != POLY_OK) return st;
        if (!ws || ws_bytes < r.total) return POLY_ERR_WORKSPACE;
        hipStream_t s = (hipStream_t)stream;
        clear_u64(at<unsigned long long>(ws, 0), 1, s);
        if (a->npolys == 0) {
            clear_u64((unsigned long long *)out->row_ptr, 1, s);
            LAUNCH_CHECK();
            return POLY_OK;
        }
        return run_mul_rows(a, b, out, zero_tol, ws, r, s);
    }
    MulPlan m;
    if ((st = plan_mul(a, b, m)) != POLY_OK) return st;
    if (!ws || ws_bytes < m.total) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t P = a->npolys;
    const int64_t Ta = total_terms(a), Tb = total_terms(b);
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0) {
        clear_u64((unsigned long long *)out->row_ptr, 1, s);
        LAUNCH_CHECK();
        return POLY_OK;
    }
    unsigned long long *queues = at<unsigned long long>(ws, m.queues);
    clear_u64(queues, 4, s);
    clear_u64(at<unsigned long long>(ws, m.cursor), 1, s);
    MulArgs A;
    A.P = P;
    A.a_rp = a->row_ptr;
    A.b_rp = b->row_ptr;
    A.a_c = a->coefs;
    A.b_c = b->coefs;
    A.ka = at<uint64_t>(ws, m.ka);
    A.kb = at<uint64_t>(ws, m.kb);
    A.ka_s = at<uint64_t>(ws, m.ka_s);
    A.kb_s = at<uint64_t>(ws, m.kb_s);
    A.perm_a = at<uint32_t>(ws, m.perm_a);
    A.perm_b = at<uint32_t>(ws, m.perm_b);
    A.ca_s = at<double>(ws, m.ca_s);
    A.cb_s = at<double>(ws, m.cb_s);
    A.pb_start = at<int64_t>(ws, m.pb_start);
    A.bk_pair = at<int32_t>(ws, m.bk_pair);
    A.bk_lo = at<uint64_t>(ws, m.bk_lo);
    A.bk_hi = at<uint64_t>(ws, m.bk_hi);
    A.bk_stage_off = at<int64_t>(ws, m.bk_stage_off);
    A.bk_count = at<int64_t>(ws, m.bk_count);
    A.stage_cursor = at<unsigned long long>(ws, m.cursor);
    A.st_key = at<uint64_t>(ws, m.st_key);
    A.st_coef = at<double>(ws, m.st_coef);
    A.tol = zero_tol;
    A.nbuckets = m.nbuckets;
    A.st_capacity = m.raw;
    A.status = status;
    hipLaunchKernelGGL(k_mul_init_buckets, dim3(grid1(m.nbuckets, 256)), dim3(256), 0, s, A);
    // the sort path orders mixed-radix keys (radix max_exp(a) + max_exp(b) + 1),
    // the bucket paths bit-field keys
    const uint64_t radix = (uint64_t)a->max_exp + (uint64_t)b->max_exp + 1;
    if (m.sort_mode) {
        if (Ta > 0)
            hipLaunchKernelGGL(k_gs_pack_radix, dim3(grid1(Ta, 256)), dim3(256), 0, s, a->exps, Ta, n, radix,
                               a->max_exp, (uint64_t *)A.ka, status);
        if (Tb > 0)
            hipLaunchKernelGGL(k_gs_pack_radix, dim3(grid1(Tb, 256)), dim3(256), 0, s, b->exps, Tb, n, radix,
                               b->max_exp, (uint64_t *)A.kb, status);
    } else {
        if (Ta > 0)
            hipLaunchKernelGGL(k_pack, dim3(grid1(Ta, 256)), dim3(256), 0, s, a->exps, Ta, n, bits, a->max_exp,
                               (uint64_t *)A.ka, status);
        if (Tb > 0)
            hipLaunchKernelGGL(k_pack, dim3(grid1(Tb, 256)), dim3(256), 0, s, b->exps, Tb, n, bits, b->max_exp,
                               (uint64_t *)A.kb, status);
    }
    int64_t *cnt_tmp = at<int64_t>(ws, m.cnt_tmp);
    if (!m.sort_mode) {
        // the bucket paths take both operands in key order
        const SegArgs sa = presort_args(a, (uint64_t *)A.ka, (uint64_t *)A.ka_s, (uint32_t *)A.perm_a, cnt_tmp,
                                        at<int64_t>(ws, m.order_a), queues + 0, s);
        const SegArgs sb = presort_args(b, (uint64_t *)A.kb, (uint64_t *)A.kb_s, (uint32_t *)A.perm_b, cnt_tmp,
                                        at<int64_t>(ws, m.order_b), queues + 1, s);
        const int64_t pgrid = std::min<int64_t>(P, (int64_t)device_cus() * tunables().seg_blocks_per_cu);
        hipLaunchKernelGGL(k_seg_sort2, dim3((unsigned)(2 * pgrid)), dim3(SEG_THREADS), 0, s, sa, sb);
        hipLaunchKernelGGL(k_mul_sorted_coefs, dim3((unsigned)P), dim3(256), 0, s, a->row_ptr, A.perm_a, a->coefs,
                           (double *)A.ca_s);
        hipLaunchKernelGGL(k_mul_sorted_coefs, dim3((unsigned)P), dim3(256), 0, s, b->row_ptr, A.perm_b, b->coefs,
                           (double *)A.cb_s);
    }
    if (m.sort_mode) {
        // ---- one pair: generate the raw product, radix sort it, merge runs
        ensure_lds_attrs();
        const int64_t R = m.raw, nb = m.gs_blocks;
        uint64_t *kcur = at<uint64_t>(ws, m.gs_keys0), *knext = at<uint64_t>(ws, m.gs_keys1);
        uint32_t *vcur = at<uint32_t>(ws, m.gs_vals0), *vnext = at<uint32_t>(ws, m.gs_vals1);
        int64_t *hist = at<int64_t>(ws, m.gs_hist), *hoff = at<int64_t>(ws, m.gs_hoff);
        int64_t *tmp = at<int64_t>(ws, m.gs_tmp);
        // scan state: cleared here for the first pass, then by each pass's
        // scatter (after its scan has finished) for the next scan
        const int64_t scan_state = scan_tmp_count(std::max<int64_t>(sort_bins() * m.gs_blocks, ceil_div(R, MG_TILE)));
        clear_u64((unsigned long long *)tmp, scan_state, s);

        // key range r^n (at most 2^(n * bits), so it fits 64 bits); as few
        // passes of at most sort_bits() bits as it needs, digits as even as possible
        unsigned __int128 span = 1;
        for (int i = 0; i < n; ++i) span *= radix;
        const uint64_t kmax = (uint64_t)(span - 1);
        const int key_bits = kmax ? 64 - __builtin_clzll((unsigned long long)kmax) : 0;
        const int passes = (key_bits + sort_bits() - 1) / sort_bits();
        const int db = std::max(passes ? (key_bits + passes - 1) / passes : GS_MIN_BITS, GS_MIN_BITS);
        // after the first pass, the digits still to sort and the raw index
        // share one 64-bit word when they fit: 8 bytes per element per pass
        // instead of 12, keys rebuilt from raw indices by the merge
        const int raw_bits = R > 1 ? 64 - __builtin_clzll((unsigned long long)(R - 1)) : 0;
        const bool packed = passes >= 2 && key_bits - db + raw_bits <= 64;
        const int64_t hgrid = std::min<int64_t>(ceil_div(nb, GS_HIST_THREADS / kWave), (int64_t)device_cus() * 8);
        // the first pass generates the raw product from the operands (keys
        // ka[i] + kb_s[j] in raw order): it is never written to memory
        GsGen gen;
        gen.ka = (const uint64_t *)A.ka;
        gen.kb = (const uint64_t *)A.kb;
        gen.tb = (uint32_t)Tb;
        gen.inv_tb = 1.0 / (double)Tb;
        auto pass = [&](auto dbc, int p) {
            constexpr int DB = decltype(dbc)::value;
            const int shift = packed && p > 0 ? raw_bits + (p - 1) * DB : p * DB;
            if (p == 0)
                hipLaunchKernelGGL((k_gs_hist<DB, true>), dim3((unsigned)hgrid), dim3(GS_HIST_THREADS), 0, s,
                                   (const uint64_t *)kcur, R, shift, nb, hist, gen);
            else
                hipLaunchKernelGGL((k_gs_hist<DB, false>), dim3((unsigned)hgrid), dim3(GS_HIST_THREADS), 0, s,
                                   (const uint64_t *)kcur, R, shift, nb, hist, gen);
            launch_scan(hist, ((int64_t)1 << DB) * nb, hoff, tmp, status, s, true);
            TimedLaunch tl(POLY_TIMING_MUL, s);
            auto scatter = [&](auto modec) {
                constexpr int MODE = decltype(modec)::value;
                hipLaunchKernelGGL((k_gs_scatter<DB, MODE>), dim3((unsigned)nb), dim3(GS_SC_THREADS), 0, s,
                                   (const uint64_t *)kcur, (const uint32_t *)vcur, R, shift, nb,
                                   (const int64_t *)hoff, knext, vnext, raw_bits, (unsigned long long *)tmp,
                                   scan_state, gen);
            };
            if (p == 0 && packed) scatter(std::integral_constant<int, GS_GEN_TO_PACKED>());
            else if (p == 0) scatter(std::integral_constant<int, GS_GEN_KV>());
            else if (packed) scatter(std::integral_constant<int, GS_PACKED>());
            else scatter(std::integral_constant<int, GS_KV>());
            tl.done(s);
        };
        if (passes == 0)   // a single key value: the raw product unsorted
            hipLaunchKernelGGL(k_gs_generate, dim3((unsigned)std::min<int64_t>(Ta, 65535)), dim3(GS_THREADS), 0, s,
                               A.ka, A.kb, Ta, Tb, kcur, vcur);
        for (int p = 0; p < passes; ++p) {
            switch (db) {
            case 4: pass(std::integral_constant<int, 4>(), p); break;
            case 5: pass(std::integral_constant<int, 5>(), p); break;
            case 6: pass(std::integral_constant<int, 6>(), p); break;
            case 7: pass(std::integral_constant<int, 7>(), p); break;
            case 8: pass(std::integral_constant<int, 8>(), p); break;
            case 9: pass(std::integral_constant<int, 9>(), p); break;
            case 10: pass(std::integral_constant<int, 10>(), p); break;
            default: pass(std::integral_constant<int, 11>(), p); break;
            }
            std::swap(kcur, knext);
            std::swap(vcur, vnext);
        }
        int64_t *cnt = at<int64_t>(ws, m.gs_count), *soff = at<int64_t>(ws, m.gs_soff);
        int64_t *ooff = at<int64_t>(ws, m.gs_ooff);
        RadixDecode dec;
        dec.radix = radix;
        dec.n = n;
        dec.bits = bits;
        dec.chunk = 1;
        dec.div = radix;
        while (dec.chunk < n && dec.div * radix <= 0xffffffffull) {
            dec.div *= radix;
            ++dec.chunk;
        }
        dec.div_magic = ~0ull / dec.div;
        dec.digit_magic = (uint32_t)(0xffffffffull / radix);
        const int64_t mb = m.gs_mblocks;
        const int64_t mgrid = std::min<int64_t>(mb, (int64_t)device_cus() * MG_BLOCKS_PER_CU);
        GsKC *pa = at<GsKC>(ws, m.gs_pa), *pb = at<GsKC>(ws, m.gs_pb);
        if (packed) {
            hipLaunchKernelGGL(k_gs_pairs, dim3(grid1(Ta, 256)), dim3(256), 0, s, (const uint64_t *)A.ka, a->coefs, Ta,
                               pa);
            hipLaunchKernelGGL(k_gs_pairs, dim3(grid1(Tb, 256)), dim3(256), 0, s, (const uint64_t *)A.kb, b->coefs,
                               Tb, pb);
            hipLaunchKernelGGL(k_gs_merge<true>, dim3((unsigned)mgrid), dim3(MG_THREADS), 0, s,
                               (const uint64_t *)kcur, (const uint32_t *)vcur, R, Ta, Tb, (const uint64_t *)A.ka,
                               (const uint64_t *)A.kb, raw_bits, a->coefs, b->coefs, (const GsKC *)pa,
                               (const GsKC *)pb, zero_tol, dec, A.st_key, A.st_coef, cnt, soff);
        } else {
            hipLaunchKernelGGL(k_gs_merge<false>, dim3((unsigned)mgrid), dim3(MG_THREADS), 0, s,
                               (const uint64_t *)kcur, (const uint32_t *)vcur, R, Ta, Tb, (const uint64_t *)A.ka,
                               (const uint64_t *)A.kb, raw_bits, a->coefs, b->coefs, (const GsKC *)pa,
                               (const GsKC *)pb, zero_tol, dec, A.st_key, A.st_coef, cnt, soff);
        }
        launch_scan(cnt, mb, ooff, tmp, status, s, true);
        hipLaunchKernelGGL(k_compact, dim3((unsigned)mb), dim3(256), 0, s, (const int64_t *)soff,
                           (const int64_t *)cnt, (const int64_t *)ooff, (const uint64_t *)A.st_key,
                           (const double *)A.st_coef, n, bits, out->exps, out->coefs, out->capacity, status);
        hipLaunchKernelGGL(k_gs_rowptr, dim3(1), dim3(64), 0, s, (const int64_t *)ooff, mb, out->row_ptr);
        LAUNCH_CHECK();
        return POLY_OK;
    }
    int64_t *pb_count = at<int64_t>(ws, m.pb_count);
    hipLaunchKernelGGL(k_mul_plan, dim3(grid1(P, 256)), dim3(256), 0, s, a->row_ptr, b->row_ptr, P, pb_count,
                       m.target);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, pb_count, P, (int64_t *)A.pb_start);
    hipLaunchKernelGGL(k_mul_splitters, dim3((unsigned)P), dim3(512), 0, s, A);
    if (m.lds_mode) {
        ensure_lds_attrs();
        TimedLaunch tl(POLY_TIMING_MUL, s);
        hipLaunchKernelGGL(k_mul_buckets_lds, dim3((unsigned)m.nbuckets), dim3(MB_THREADS), m.lds_dyn, s, A);
        tl.done(s);
    } else {
        hipLaunchKernelGGL(k_mul_buckets, dim3((unsigned)m.nbuckets), dim3(MUL_THREADS), 0, s, A);
    }
    int64_t *out_off = at<int64_t>(ws, m.out_off);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, A.bk_count, m.nbuckets, out_off);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)m.nbuckets), dim3(256), 0, s, A.bk_stage_off, A.bk_count,
                       out_off, A.st_key, A.st_coef, n, bits, out->exps, out->coefs, out->capacity, status);
    hipLaunchKernelGGL(k_mul_rowptr, dim3(grid1(P + 1, 256)), dim3(256), 0, s, out_off, A.pb_start, P,
                       out->row_ptr, m.nbuckets);
    LAUNCH_CHECK();
    return POLY_OK;
}

// ------------------------------------------------------------------ jacobian

poly_status poly_jacobian_workspace(const poly_csr *in, size_t *ws_bytes)
{
    poly_status st = check_csr(in, true);
    if (st != POLY_OK) return st;
    if (!ws_bytes) return POLY_ERR_ARG;
    Layout L;
    plan_form(in, in->nvars, L);
    *ws_bytes = L.total();
    return POLY_OK;
}

poly_status poly_jacobian(const poly_csr *in, poly_csr *out, void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_csr(in, true);
    if (st != POLY_OK) return st;
    if ((st = check_csr(out, false)) != POLY_OK) return st;
    const int n = in->nvars;
    const int64_t P = in->npolys;
    if (out->nvars != n || out->npolys != P * n) return POLY_ERR_ARG;
    Layout L;
    const FormPlan fp = plan_form(in, n, L);
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0) {
        clear_u64((unsigned long long *)out->row_ptr, 1, s);
        LAUNCH_CHECK();
        return POLY_OK;
    }
    FormArgs F = form_args(in->row_ptr, in->exps, in->coefs, n, 0, 0, status, (int32_t)POLY_ERR_CAPACITY);
    F.out_rp = out->row_ptr;
    F.out_exps = out->exps;
    F.out_coefs = out->coefs;
    F.capacity = out->capacity;
    run_form(fp, F, ws, s);
    LAUNCH_CHECK();
    return POLY_OK;
}

// ---------------------------------------------------------------------- eval

static poly_status check_eval(const poly_csr *f, const double *X, int64_t N, const void *out)
{
    poly_status st = check_csr(f, true);
    if (st != POLY_OK) return st;
    if (N < 0) return POLY_ERR_ARG;
    if (N > 0 && f->npolys > 0 && (!X || !out)) return POLY_ERR_ARG;
    return POLY_OK;
}

// ------------------------------------------------ split precision (CSR)
//
// prec = POLY_SPLIT_BF16 on the sparse entry points: the batch must be a
// shared monomial set stored as CSR -- every polynomial holds the same K
// exponent rows in the same order (equal row lengths, checked on the host;
// equal rows, checked on the device: POLY_ERR_UNSUPPORTED otherwise).  Its
// coefficients are then the row-major P x K matrix of the dense
// contraction, used in place; derivatives are contractions over derived
// bases (e - u_j, coefficients m c with the integer multiplier m).

namespace {

struct SplitCsrPlan {
    int64_t K = 0;
    size_t dense = 0, dbasis = 0, dC = 0, total = 0;
};

static poly_status plan_split_csr(const poly_csr *f, int64_t N, int32_t nslices, bool derived, SplitCsrPlan &sp)
{
    const int64_t P = f->npolys;
    sp.K = P > 0 ? f->row_ptr_host[1] : 0;
    for (int64_t p = 1; p <= P; ++p)
        if (f->row_ptr_host[p] - f->row_ptr_host[p - 1] != sp.K) return POLY_ERR_UNSUPPORTED;
    size_t dws = 0;
    poly_status st = dense_workspace(f->nvars, sp.K, P, N, POLY_SPLIT_BF16, nslices, &dws);
    if (st != POLY_OK) return st;
    Layout L;
    L.off = std::max(dws, (size_t)kWsHeadBytes);
    sp.dense = 0;   // the dense path's workspace starts at ws (its status word is the call's)
    if (derived) {
        sp.dbasis = L.take((size_t)sp.K * f->nvars);
        sp.dC = L.take(8 * (size_t)P * sp.K);
    }
    sp.total = L.total();
    return POLY_OK;
}

// mode 0: values; 1: gradient G[p][pt][j]; 2: Hessian H[p][pt][j][k]
static poly_status run_split_csr(int mode, const poly_csr *f, const double *X, int64_t N, double *out, int32_t nslices,
                          void *ws, size_t ws_bytes, hipStream_t s)
{
    SplitCsrPlan sp;
    poly_status st = plan_split_csr(f, N, nslices, mode != 0, sp);
    if (st != POLY_OK) return st;
    if (!ws || ws_bytes < sp.total) return POLY_ERR_WORKSPACE;
    const int n = f->nvars;
    const int64_t P = f->npolys, K = sp.K;
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0 || N == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    if (mode == 0) {
        st = dense_run(n, K, f->exps, f->max_exp, P, f->coefs, N, X, out, POLY_SPLIT_BF16, nslices, ws, ws_bytes, s,
                       1);
    } else {
        uint8_t *db = at<uint8_t>(ws, sp.dbasis);
        double *dC = at<double>(ws, sp.dC);
        const unsigned g = (unsigned)std::min<int64_t>(grid1(P * K, 256), 65535);
        for (int j = 0; j < n && st == POLY_OK; ++j) {
            for (int k = (mode == 1 ? -1 : j); k < (mode == 1 ? 0 : n) && st == POLY_OK; ++k) {
                hipLaunchKernelGGL(k_derive_basis, dim3(g), dim3(256), 0, s, f->exps, K, n, j, k, db, f->coefs, P, dC);
                double *dst = mode == 1 ? out + j : out + (int64_t)j * n + k;
                st = dense_run(n, K, db, f->max_exp, P, dC, N, X, dst, POLY_SPLIT_BF16, nslices, ws, ws_bytes, s,
                               mode == 1 ? n : (int64_t)n * n);
            }
        }
        if (st == POLY_OK && mode == 2)
            hipLaunchKernelGGL(k_hess_mirror, dim3((unsigned)std::min<int64_t>(grid1(P * N * n * n, 256), 65535)),
                               dim3(256), 0, s, out, P * N, n);
    }
    if (st != POLY_OK) return st;
    // every polynomial must list polynomial 0's rows (checked after the
    // contractions, which clear the status word first)
    if (P > 1 && K > 0)
        hipLaunchKernelGGL(k_check_shared, dim3((unsigned)std::min<int64_t>(grid1((P - 1) * K * n, 256), 65535)),
                           dim3(256), 0, s, f->exps, P, K, n, status);
    LAUNCH_CHECK();
    return POLY_OK;
}

static poly_status split_csr_workspace(int mode, const poly_csr *f, int64_t N, int32_t nslices, size_t *ws_bytes)
{
    SplitCsrPlan sp;
    poly_status st = plan_split_csr(f, N, nslices, mode != 0, sp);
    if (st != POLY_OK) return st;
    *ws_bytes = sp.total;
    return POLY_OK;
}

}  // namespace

poly_status poly_eval_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes)
{
    poly_status st = check_eval(f, nullptr, 0, nullptr);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    if (prec == POLY_SPLIT_BF16) return split_csr_workspace(0, f, N, nslices, ws_bytes);
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    Layout L;
    L.take(16 * total_terms(f));
    L.take(eval_partial_bytes(f->npolys, N, eval_segments(f->npolys, N, total_terms(f))));
    *ws_bytes = L.total();
    return POLY_OK;
}

poly_status poly_eval(const poly_csr *f, const double *X, int64_t N, double *Y, poly_prec prec, int32_t nslices,
                      void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_eval(f, X, N, Y);
    if (st != POLY_OK) return st;
    if (prec == POLY_SPLIT_BF16) {
        ensure_lds_attrs();
        return run_split_csr(0, f, X, N, Y, nslices, ws, ws_bytes, (hipStream_t)stream);
    }
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    const int64_t T = total_terms(f);
    Layout L;
    const size_t o_enc = L.take(16 * T);
    const int64_t S = eval_segments(f->npolys, N, T);
    const size_t o_part = L.take(eval_partial_bytes(f->npolys, N, S));
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (f->npolys == 0 || N == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    uint32_t *enc = at<uint32_t>(ws, o_enc);
    // small calls take the general kernel alone (one launch): the degree class
    // pays only where the evaluation itself is long
    uint32_t *md = T * N >= ((int64_t)1 << 22) ? ws_maxdeg(ws) : nullptr;
    if (T > 0) hipLaunchKernelGGL(k_encode_factors, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, f->nvars, enc,
                                  (const int64_t *)nullptr, md);
    EvalArgs A;
    memset(&A, 0, sizeof(A));
    A.maxdeg = md;
    A.rp = f->row_ptr;
    A.exps = f->exps;
    A.coefs = f->coefs;
    A.n = f->nvars;
    A.X = X;
    A.N = N;
    A.Q = f->npolys;
    A.mode = OUT_EVAL;
    A.Y = Y;
    A.term_limit = T;
    launch_eval_blocks(A, enc, at<double>(ws, o_part), S, s);
    LAUNCH_CHECK();
    return POLY_OK;
}

poly_status poly_grad_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes)
{
    poly_status st = check_eval(f, nullptr, 0, nullptr);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    if (prec == POLY_SPLIT_BF16) return split_csr_workspace(1, f, N, nslices, ws_bytes);
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    Layout L;
    plan_grad(f, N, L);
    *ws_bytes = L.total();
    return POLY_OK;
}

poly_status poly_grad(const poly_csr *f, const double *X, int64_t N, double *G, poly_prec prec, int32_t nslices,
                      void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_eval(f, X, N, G);
    if (st != POLY_OK) return st;
    if (prec == POLY_SPLIT_BF16) {
        ensure_lds_attrs();
        return run_split_csr(1, f, X, N, G, nslices, ws, ws_bytes, (hipStream_t)stream);
    }
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    Layout L;
    const GradPlan g = plan_grad(f, N, L);
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (f->npolys == 0 || N == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    return run_grad(f, X, N, G, ws, g, s);
}

// Hessian: the Jacobian with original coefficients, then the entries (j, k),
// j <= k, formed from it (mode 1), encoded and evaluated in one pass.
struct HessPlan {
    FormPlan jform, hform;
    size_t jrp, jexps, jcoefs, hrp, hexps, hcoefs, henc, part, stage;
    int64_t jcap, hcap, S;
};

static HessPlan plan_hess(const poly_csr *f, int64_t N, Layout &L)
{
    HessPlan h;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    const int64_t npairs = (int64_t)n * (n + 1) / 2;
    h.jcap = grad_terms_bound(T, n);
    h.hcap = hess_terms_bound(T, npairs);
    h.jform = plan_form(f, n, L);
    h.jrp = L.take(8 * (P * n + 1));
    h.jexps = L.take((size_t)h.jcap * n);
    h.jcoefs = L.take(8 * h.jcap);
    h.hform = plan_form_bound(P * n, h.jcap, n, L);
    h.hrp = L.take(8 * (P * n * n + 1));
    h.hexps = L.take((size_t)h.hcap * n);
    h.hcoefs = L.take(8 * h.hcap);
    h.henc = L.take(16 * h.hcap);
    h.S = eval_segments(P * n * n, N, T);
    h.part = L.take(eval_partial_bytes(P * n * n, N, h.S));
    h.stage = L.take(8 * (size_t)P * n * n * N);   // entries (j <= k), point-contiguous
    return h;
}

poly_status poly_hess_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes)
{
    poly_status st = check_eval(f, nullptr, 0, nullptr);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    if (prec == POLY_SPLIT_BF16) return split_csr_workspace(2, f, N, nslices, ws_bytes);
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    Layout L;
    plan_hess(f, N, L);
    *ws_bytes = L.total();
    return POLY_OK;
}

static poly_status run_hess(const poly_csr *f, const double *X, int64_t N, double *H, void *ws, const HessPlan &h,
                     hipStream_t s)
{
    const int n = f->nvars;
    const int64_t P = f->npolys;
    int32_t *status = at<int32_t>(ws, 0);
    int64_t *jrp = at<int64_t>(ws, h.jrp);
    uint8_t *jexps = at<uint8_t>(ws, h.jexps);
    double *jcoefs = at<double>(ws, h.jcoefs);
    int64_t *hrp = at<int64_t>(ws, h.hrp);
    uint8_t *hexps = at<uint8_t>(ws, h.hexps);
    double *hcoefs = at<double>(ws, h.hcoefs);
    uint32_t *henc = at<uint32_t>(ws, h.henc);
    FormArgs J = form_args(f->row_ptr, f->exps, f->coefs, n, 0, 1, status, (int32_t)POLY_ERR_WORKSPACE);
    J.out_rp = jrp;
    J.out_exps = jexps;
    J.out_coefs = jcoefs;
    J.capacity = h.jcap;
    run_form(h.jform, J, ws, s);
    FormArgs F = form_args(jrp, jexps, jcoefs, n, 1, 0, status, (int32_t)POLY_ERR_WORKSPACE);
    F.out_rp = hrp;
    F.out_exps = hexps;
    F.out_coefs = hcoefs;
    F.capacity = h.hcap;
    run_form(h.hform, F, ws, s);
    hipLaunchKernelGGL(k_encode_factors, dim3(grid1(h.hcap, 256)), dim3(256), 0, s, hexps, h.hcap, n, henc,
                       (const int64_t *)(hrp + P * n * n), ws_maxdeg(ws));
    EvalArgs A;
    memset(&A, 0, sizeof(A));
    A.maxdeg = ws_maxdeg(ws);
    A.rp = hrp;
    A.exps = hexps;
    A.coefs = hcoefs;
    A.n = n;
    A.X = X;
    A.N = N;
    A.Q = P * n * n;
    A.mode = OUT_HESS;
    A.Y = at<double>(ws, h.stage);
    A.term_limit = h.hcap;
    launch_eval_blocks(A, henc, at<double>(ws, h.part), h.S, s);
    hipLaunchKernelGGL(k_hess_transpose, dim3((unsigned)ceil_div(N, 32), (unsigned)n,
                                               (unsigned)std::min<int64_t>(P, 65535)), dim3(256),
                       (size_t)n * 33 * sizeof(double), s, (const double *)A.Y, P, N, n, H);
    LAUNCH_CHECK();
    return POLY_OK;
}

poly_status poly_hess(const poly_csr *f, const double *X, int64_t N, double *H, poly_prec prec, int32_t nslices,
                      void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_eval(f, X, N, H);
    if (st != POLY_OK) return st;
    if (prec == POLY_SPLIT_BF16) {
        ensure_lds_attrs();
        return run_split_csr(2, f, X, N, H, nslices, ws, ws_bytes, (hipStream_t)stream);
    }
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    Layout L;
    const HessPlan h = plan_hess(f, N, L);
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (f->npolys == 0 || N == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    return run_hess(f, X, N, H, ws, h, s);
}

// ------------------------------------------------------------ affine normal

// The gradient and Hessian paths, then one workgroup per point.
struct AffinePlan {
    GradPlan g;
    HessPlan h;
    size_t G, H, enc;
};

static AffinePlan plan_affine(const poly_csr *f, int64_t N, Layout &L)
{
    AffinePlan a;
    const int n = f->nvars;
    a.g = plan_grad(f, N, L);
    a.h = plan_hess(f, N, L);
    a.G = L.take(8 * (size_t)N * n);
    a.H = L.take(8 * (size_t)N * n * n);
    a.enc = L.take(16 * (size_t)std::max<int64_t>(total_terms(f), 1));
    return a;
}

static poly_status check_affine(const poly_csr *f, const double *X, int64_t N, const double *D, double reg)
{
    poly_status st = check_eval(f, X, N, D);
    if (st != POLY_OK) return st;
    if (f->npolys != 1 || f->nvars < 2 || f->nvars > AN_MAX_N || !(reg >= 0.0) || reg > 1e300)
        return f->nvars > AN_MAX_N ? POLY_ERR_UNSUPPORTED : POLY_ERR_ARG;
    return POLY_OK;
}

namespace {

// Products of polynomial matrices: the raw batch (sizes and offsets from
// the row pointers, then one workgroup per output entry), then the batched
// simplify.  The simplify workspace comes first; the raw batch after it.
// When an output entry has at least simplify_wide_min raw terms, the raw
// products are written as device-wide simplify keys instead (one thread per
// raw term, operand monomials packed once).
struct MtimesPlan {
    SimplifyPlan sp;
    WidePlan wide;
    size_t rrp, re, rc, sizes, tmp, ka, kb, total;
    int64_t raw;
    int bits;
};

static poly_status check_mtimes(const poly_csr *A, const poly_csr *B, int64_t I, int64_t K, int64_t J)
{
    poly_status st;
    if ((st = check_csr(A, true)) != POLY_OK) return st;
    if ((st = check_csr(B, true)) != POLY_OK) return st;
    if (I < 0 || K < 0 || J < 0 || A->nvars != B->nvars || A->npolys != I * K || B->npolys != K * J)
        return POLY_ERR_ARG;
    if (A->max_exp + B->max_exp > 255) return POLY_ERR_ARG;
    return POLY_OK;
}

static poly_status plan_mtimes(const poly_csr *A, const poly_csr *B, int64_t I, int64_t K, int64_t J,
                        std::vector<int64_t> &rph, MtimesPlan &m)
{
    const int64_t Q = I * J;
    rph.assign(Q + 1, 0);
    for (int64_t i = 0; i < I; ++i)
        for (int64_t j = 0; j < J; ++j) {
            int64_t r = 0;
            for (int64_t k = 0; k < K; ++k)
                r += (A->row_ptr_host[i * K + k + 1] - A->row_ptr_host[i * K + k]) *
                     (B->row_ptr_host[k * J + j + 1] - B->row_ptr_host[k * J + j]);
            rph[i * J + j + 1] = rph[i * J + j] + r;
        }
    m.raw = rph[Q];
    if (m.raw >= (int64_t(1) << 32)) return POLY_ERR_UNSUPPORTED;
    m.bits = bit_width_u32((uint32_t)(A->max_exp + B->max_exp));
    const uint32_t radix = (uint32_t)(A->max_exp + B->max_exp) + 1;
    Layout L;
    const bool fields = (int64_t)A->nvars * m.bits <= 64;
    if (fields && wide_wanted(Q, m.raw, max_segment(rph.data(), Q), A->nvars, radix)) {
        plan_wide(m.wide, L, Q, m.raw, A->nvars, radix);
        m.ka = L.take(8 * total_terms(A));
        m.kb = L.take(8 * total_terms(B));
        m.re = 0;
    } else {
        m.sp = plan_simplify(Q, m.raw, rph.data(), A->nvars, radix);
        if (!m.sp.ok) return POLY_ERR_UNSUPPORTED;
        L.off = m.sp.total;
        m.re = L.take((size_t)m.raw * A->nvars);
        m.ka = m.kb = 0;
    }
    m.rrp = L.take(8 * (Q + 1));
    m.rc = L.take(8 * m.raw);
    m.sizes = L.take(8 * Q);
    m.tmp = L.take(8 * scan_tmp_count(Q));
    m.total = L.total();
    return POLY_OK;
}

}  // namespace

poly_status poly_mtimes_workspace(const poly_csr *A, const poly_csr *B, int64_t I, int64_t K, int64_t J,
                                  size_t *ws_bytes, int64_t *raw_terms)
{
    poly_status st = check_mtimes(A, B, I, K, J);
    if (st != POLY_OK) return st;
    if (!ws_bytes || !raw_terms) return POLY_ERR_ARG;
    std::vector<int64_t> rph;
    MtimesPlan m;
    if ((st = plan_mtimes(A, B, I, K, J, rph, m)) != POLY_OK) return st;
    *ws_bytes = m.total;
    *raw_terms = m.raw;
    return POLY_OK;
}

poly_status poly_mtimes(const poly_csr *A, const poly_csr *B, int64_t I, int64_t K, int64_t J, poly_csr *out,
                        double zero_tol, void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_mtimes(A, B, I, K, J);
    if (st != POLY_OK) return st;
    if ((st = check_csr(out, false)) != POLY_OK) return st;
    const int n = A->nvars;
    if (out->nvars != n || out->npolys != I * J || out->max_exp < A->max_exp + B->max_exp) return POLY_ERR_ARG;
    if (!(zero_tol >= 0.0)) return POLY_ERR_ARG;
    std::vector<int64_t> rph;
    MtimesPlan m;
    if ((st = plan_mtimes(A, B, I, K, J, rph, m)) != POLY_OK) return st;
    if (!ws || ws_bytes < m.total) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    const int64_t Q = I * J;
    if (Q == 0) {
        clear_u64((unsigned long long *)out->row_ptr, 1, s);
        LAUNCH_CHECK();
        return POLY_OK;
    }
    int64_t *sizes = at<int64_t>(ws, m.sizes);
    int64_t *rrp = at<int64_t>(ws, m.rrp);
    uint8_t *re = at<uint8_t>(ws, m.re);
    double *rc = at<double>(ws, m.rc);
    hipLaunchKernelGGL(k_mat_raw_sizes, dim3(grid1(Q, 256)), dim3(256), 0, s, A->row_ptr, B->row_ptr, I, K, J, sizes);
    launch_scan(sizes, Q, rrp, at<int64_t>(ws, m.tmp), status, s);
    if (m.wide.on) {
        const int64_t TA = total_terms(A), TB = total_terms(B);
        uint64_t *ka = at<uint64_t>(ws, m.ka), *kb = at<uint64_t>(ws, m.kb);
        const uint64_t radix = m.wide.radix;
        if (TA > 0)
            hipLaunchKernelGGL(k_gs_pack_radix, dim3(grid1(TA, 256)), dim3(256), 0, s, A->exps, TA, n, radix,
                               A->max_exp, ka, status);
        if (TB > 0)
            hipLaunchKernelGGL(k_gs_pack_radix, dim3(grid1(TB, 256)), dim3(256), 0, s, B->exps, TB, n, radix,
                               B->max_exp, kb, status);
        hipLaunchKernelGGL(k_mat_keys, dim3(grid1(m.raw, 256)), dim3(256), 0, s, A->row_ptr, (const uint64_t *)ka,
                           A->coefs, B->row_ptr, (const uint64_t *)kb, B->coefs, I, K, J, (const int64_t *)rrp,
                           m.raw, m.wide.span, at<uint64_t>(ws, m.wide.keys0), at<uint32_t>(ws, m.wide.vals0), rc);
        return run_wide(m.wide, ws, Q, m.raw, n, m.bits, rc, zero_tol, out, s);
    }
    hipLaunchKernelGGL(k_mat_expand, dim3((unsigned)Q), dim3(MAT_THREADS), 0, s, A->row_ptr, A->exps, A->coefs,
                       B->row_ptr, B->exps, B->coefs, I, K, J, n, (const int64_t *)rrp, re, rc);
    poly_csr R;
    R.nvars = n;
    R.max_exp = A->max_exp + B->max_exp;
    R.npolys = Q;
    R.capacity = m.raw;
    R.row_ptr_host = rph.data();
    R.row_ptr = rrp;
    R.exps = re;
    R.coefs = rc;
    return run_simplify(&R, out, zero_tol, ws, m.sp, s);
}

poly_status poly_concat(const poly_csr *const *ins, int32_t nin, poly_csr *out, void *stream)
{
    if (nin < 0 || (nin > 0 && !ins)) return POLY_ERR_ARG;
    poly_status st = check_csr(out, false);
    if (st != POLY_OK) return st;
    int64_t P = 0, T = 0;
    for (int32_t i = 0; i < nin; ++i) {
        if ((st = check_csr(ins[i], true)) != POLY_OK) return st;
        if (ins[i]->nvars != out->nvars || ins[i]->max_exp > out->max_exp) return POLY_ERR_ARG;
        P += ins[i]->npolys;
        T += total_terms(ins[i]);
    }
    if (out->npolys != P) return POLY_ERR_ARG;
    if (T > out->capacity) return POLY_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    clear_u64((unsigned long long *)out->row_ptr, 1, s);   // row_ptr[0] = 0, also when nothing is copied
    const int n = out->nvars;
    int64_t eo = 0, to = 0;
    for (int32_t i = 0; i < nin; ++i) {
        const poly_csr *c = ins[i];
        const int64_t Ti = total_terms(c);
        const int64_t work = std::max<int64_t>(c->npolys + 1, Ti * n);
        hipLaunchKernelGGL(k_concat_copy, dim3(std::min<unsigned>(grid1(work, 256), 4096u)), dim3(256), 0, s,
                           (const int64_t *)c->row_ptr, c->exps, c->coefs, c->npolys, Ti, n, eo, to, out->row_ptr,
                           out->exps, out->coefs);
        eo += c->npolys;
        to += Ti;
    }
    LAUNCH_CHECK();
    return POLY_OK;
}

poly_status poly_affine_normal_workspace(const poly_csr *f, int64_t N, size_t *ws_bytes)
{
    poly_status st = check_affine(f, nullptr, 0, nullptr, 0.0);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    Layout L;
    plan_affine(f, N, L);
    *ws_bytes = L.total();
    return POLY_OK;
}

poly_status poly_affine_normal(const poly_csr *f, const double *X, int64_t N, double reg, double *D, double *gnorm,
                               void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_affine(f, X, N, D, reg);
    if (st != POLY_OK) return st;
    Layout L;
    const AffinePlan a = plan_affine(f, N, L);
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (N == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    const int n = f->nvars;
    const int64_t T = total_terms(f);
    double *G = at<double>(ws, a.G);
    double *H = at<double>(ws, a.H);
    uint32_t *enc = at<uint32_t>(ws, a.enc);
    if ((st = run_grad(f, X, N, G, ws, a.g, s)) != POLY_OK) return st;
    if ((st = run_hess(f, X, N, H, ws, a.h, s)) != POLY_OK) return st;
    if (T > 0)
        hipLaunchKernelGGL(k_encode_factors, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, enc,
                           (const int64_t *)nullptr, (uint32_t *)nullptr);
    TimedLaunch tl(POLY_TIMING_AFFINE, s);
    hipLaunchKernelGGL(k_affine_normal, dim3((unsigned)N), dim3(AN_THREADS), affine_lds_bytes(n), s, n,
                       (const uint4 *)enc, f->coefs, T, X, (const double *)G, H, reg, D, gnorm,
                       status);
    tl.done(s);
    LAUNCH_CHECK();
    return POLY_OK;
}

// Probes solved at once by the stochastic route: the smallest power of two
// holding all q probes, at most AS_MAX_SLOTS, halved until the point's
// vectors fit the LDS budget (n <= 255 always fits one slot).
static int affine_stochastic_slots(int n, int q)
{
    int b = 1;
    while (b < q && b < AS_MAX_SLOTS) b <<= 1;
    while (b > 1 && affine_stochastic_lds_bytes(n, b) > AS_LDS_BUDGET) b >>= 1;
    return b;
}

poly_status poly_affine_normal_stochastic_workspace(const poly_csr *f, int64_t N, size_t *ws_bytes)
{
    poly_status st = check_affine(f, nullptr, 0, nullptr, 0.0);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    *ws_bytes = kWsHeadBytes + 16 * (size_t)std::max<int64_t>(total_terms(f), 1);
    return POLY_OK;
}

poly_status poly_affine_normal_stochastic(const poly_csr *f, const double *X, int64_t N, const double *Z, int32_t q,
                                          int32_t per_point, double reg, double tol, int32_t maxit, double *D,
                                          double *gnorm, int32_t *hv_evals, void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_affine(f, X, N, D, reg);
    if (st != POLY_OK) return st;
    if (q < 1 || (N > 0 && !Z) || (per_point != 0 && per_point != 1) || !(tol >= 0.0) || maxit < 0 ||
        N > INT32_MAX || (N > 0 && !gnorm))
        return POLY_ERR_ARG;
    if (((int64_t)q + 1) * maxit + 1 > INT32_MAX) return POLY_ERR_ARG;   // hv_evals must fit int32
    size_t need = 0;
    (void)poly_affine_normal_stochastic_workspace(f, N, &need);
    if (!ws || ws_bytes < need) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (N == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    const int n = f->nvars;
    const int64_t T = total_terms(f);
    uint32_t *enc = at<uint32_t>(ws, kWsHeadBytes);
    if (T > 0)
        hipLaunchKernelGGL(k_encode_factors, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, enc,
                           (const int64_t *)nullptr, (uint32_t *)nullptr);
    AffStochArgs A;
    A.n = n;
    A.enc = (const uint4 *)enc;
    A.coefs = f->coefs;
    A.T = T;
    A.X = X;
    A.Z = Z;
    A.per_point = per_point;
    A.q = q;
    A.slots = affine_stochastic_slots(n, q);
    A.reg = reg;
    A.tol = tol;
    A.maxit = maxit;
    A.D = D;
    A.gnorm = gnorm;
    A.hv = hv_evals;
    A.status = status;
    TimedLaunch tl(POLY_TIMING_AFFINE, s);
    hipLaunchKernelGGL(k_affine_stochastic, dim3((unsigned)N), dim3(AS_THREADS),
                       affine_stochastic_lds_bytes(n, A.slots), s, A);
    tl.done(s);
    LAUNCH_CHECK();
    return POLY_OK;
}

namespace {

// Reverse mode of eval: dX from the weighted derivative stream over the
// source terms (n up to the deriv_fused_max_n tunable) or over the formed
// Jacobian (k_eval_wsum); neither stores per-polynomial gradients.  dC from
// the support encoding over point chunks.
struct BackwardPlan {
    bool fused = false;
    size_t fenc = 0;        // factor lists (fused dX)
    DerivPlan dv;
    GradPlan g;             // dX from the formed Jacobian
    size_t senc = 0, part = 0;   // dC
    int cp = 0;
    int64_t nchunks = 0;
};

static BackwardPlan plan_backward(const poly_csr *f, int64_t N, Layout &L)
{
    BackwardPlan b;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    if (n <= tunables().deriv_fused_max_n && deriv_shape(DM_DX, n).ok) {
        b.fused = true;
        b.fenc = L.take(16 * T);
        b.dv = plan_deriv(DM_DX, n, P, T, N, L);
    } else {
        b.g = plan_grad_formed(f, N, L, true);
    }
    b.senc = L.take(16 * T);   // factor lists of the dC kernel
    b.cp = std::max(1, std::min(BWC_POINTS, 8192 / (n + 1)));
    b.nchunks = ceil_div(N, b.cp);
    b.part = L.take(8 * T * b.nchunks);
    return b;
}

// Reverse mode of the reverse mode: cotangents u (of dX) and w (of dC).
struct Backward2Plan {
    size_t fenc = 0, senc = 0, part = 0;
    DerivPlan hvp, dx, dird;
    int cp = 0;
    int64_t nchunks = 0;
};

static Backward2Plan plan_backward2(const poly_csr *f, int64_t N, Layout &L)
{
    Backward2Plan b;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    b.fenc = L.take(16 * T);
    b.hvp = plan_deriv(DM_HVP, n, P, T, N, L);
    b.dx = plan_deriv(DM_DX, n, P, T, N, L);
    b.dird = plan_deriv(DM_DIRD, n, P, T, N, L);
    b.senc = L.take(16 * T);
    b.cp = std::max(1, std::min(BWC_POINTS, 4096 / n));
    b.nchunks = ceil_div(N, b.cp);
    b.part = L.take(8 * T * b.nchunks);
    return b;
}

// dC[t] = sum_pt gY[p(t)][pt] m_t(x_pt) over point chunks, then in chunk order
static void launch_dc(const poly_csr *f, const double *X, int64_t N, const double *gY, double *dC, uint64_t *senc,
               double *part, int cp, int64_t nchunks, hipStream_t s)
{
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    if (T <= 0) return;
    if (N == 0) {
        clear_u64((unsigned long long *)dC, T, s);
        return;
    }
    hipLaunchKernelGGL(k_encode_factors, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, (uint32_t *)senc,
                       (const int64_t *)nullptr, (uint32_t *)nullptr);
    const size_t lds = (size_t)cp * (n + 1) * sizeof(double);
    hipLaunchKernelGGL(k_backward_dc, dim3(grid1(T, BWC_TERMS * BWC_THREADS), (unsigned)nchunks), dim3(BWC_THREADS),
                       lds, s, f->row_ptr, P, f->exps, n, T, X, N, gY, part, nchunks, (const uint4 *)senc, cp);
    hipLaunchKernelGGL(k_backward_dc_reduce, dim3(grid1(T, 256)), dim3(256), 0, s, (const double *)part, T, nchunks,
                       dC);
}

}  // namespace

namespace {

// prec = POLY_SPLIT_BF16 on the reverse mode: a shared monomial set stored
// as CSR (as for the forward) runs the dense reverse mode on the split
// scheme; K = the common row length, or -1 if they differ
static int64_t shared_row_length(const poly_csr *f)
{
    const int64_t P = f->npolys;
    const int64_t K = P > 0 ? f->row_ptr_host[1] : 0;
    for (int64_t p = 1; p <= P; ++p)
        if (f->row_ptr_host[p] - f->row_ptr_host[p - 1] != K) return -1;
    return K;
}

}  // namespace

poly_status poly_eval_backward_workspace(const poly_csr *f, int64_t N, poly_prec prec, int32_t nslices, size_t *ws_bytes)
{
    poly_status st = check_eval(f, nullptr, 0, nullptr);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    if (prec == POLY_SPLIT_BF16) {
        const int64_t K = shared_row_length(f);
        if (K < 0) return POLY_ERR_UNSUPPORTED;
        return dense_bwd_workspace(f->nvars, K, f->npolys, N, prec, nslices, ws_bytes);
    }
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    Layout L;
    plan_backward(f, N, L);
    *ws_bytes = L.total();
    return POLY_OK;
}

poly_status poly_eval_backward(const poly_csr *f, const double *X, int64_t N, const double *gY, double *dX,
                               double *dC, poly_prec prec, int32_t nslices, void *ws, size_t ws_bytes, void *stream)
{
    poly_status st = check_eval(f, X, N, gY);
    if (st != POLY_OK) return st;
    if (prec == POLY_SPLIT_BF16) {
        const int64_t K = shared_row_length(f);
        if (K < 0) return POLY_ERR_UNSUPPORTED;
        hipStream_t s = (hipStream_t)stream;
        st = dense_bwd_run(f->nvars, K, f->exps, f->max_exp, f->npolys, f->coefs, N, X, gY, dC, dX, prec, nslices,
                           ws, ws_bytes, s);
        if (st != POLY_OK) return st;
        // every polynomial must list polynomial 0's rows (the dense run
        // cleared the status word first)
        if (f->npolys > 1 && K > 0)
            hipLaunchKernelGGL(k_check_shared,
                               dim3((unsigned)std::min<int64_t>(grid1((f->npolys - 1) * K * f->nvars, 256), 65535)),
                               dim3(256), 0, s, f->exps, f->npolys, K, f->nvars, at<int32_t>(ws, 0));
        LAUNCH_CHECK();
        return POLY_OK;
    }
    if (prec != POLY_FP64) return POLY_ERR_ARG;
    (void)nslices;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    Layout L;
    const BackwardPlan b = plan_backward(f, N, L);
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    if (dX && N > 0) {
        if (b.fused) {
            uint64_t *enc = at<uint64_t>(ws, b.fenc);
            if (T > 0)
                hipLaunchKernelGGL(k_encode_support, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, enc,
                                   (const int64_t *)nullptr);
            DerivArgs A = deriv_args(f, enc, X, N, dX);
            A.gY = gY;
            launch_deriv<DM_DX>(A, b.dv, ws, s);
        } else {
            st = run_wsum(f, X, N, gY, dX, ws, b.g, s);
            if (st != POLY_OK) return st;
        }
    }
    if (dC) launch_dc(f, X, N, gY, dC, at<uint64_t>(ws, b.senc), at<double>(ws, b.part), b.cp, b.nchunks, s);
    LAUNCH_CHECK();
    return POLY_OK;
}

static poly_status check_backward2(const poly_csr *f, const double *X, int64_t N, const double *gY)
{
    poly_status st = check_eval(f, X, N, gY);
    if (st != POLY_OK) return st;
    if (!deriv_shape(DM_HVP, f->nvars).ok || !deriv_shape(DM_DIRD, f->nvars).ok) return POLY_ERR_UNSUPPORTED;
    return POLY_OK;
}

poly_status poly_eval_backward2_workspace(const poly_csr *f, int64_t N, size_t *ws_bytes)
{
    poly_status st = check_backward2(f, nullptr, 0, nullptr);
    if (st != POLY_OK) return st;
    if (!ws_bytes || N < 0) return POLY_ERR_ARG;
    Layout L;
    plan_backward2(f, N, L);
    *ws_bytes = L.total();
    return POLY_OK;
}

poly_status poly_eval_backward2(const poly_csr *f, const double *X, int64_t N, const double *gY, const double *u,
                                const double *w, double *ggY, double *ggX, double *ggC, void *ws, size_t ws_bytes,
                                void *stream)
{
    poly_status st = check_backward2(f, X, N, gY);
    if (st != POLY_OK) return st;
    const int n = f->nvars;
    const int64_t P = f->npolys, T = total_terms(f);
    if (T > 0 && (ggX || ggY) && !f->coefs) return POLY_ERR_ARG;
    Layout L;
    const Backward2Plan b = plan_backward2(f, N, L);
    if (!ws || ws_bytes < L.total()) return POLY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0) {
        LAUNCH_CHECK();
        return POLY_OK;
    }
    uint64_t *enc = at<uint64_t>(ws, b.fenc);
    if (T > 0 && N > 0 && (ggX || ggY))
        hipLaunchKernelGGL(k_encode_support, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, enc,
                           (const int64_t *)nullptr);
    if (ggX && N > 0) {
        DerivArgs A = deriv_args(f, enc, X, N, ggX);
        A.gY = gY;
        if (u) {   // c_t u . Hess m_t + w_t grad m_t, weighted by gY
            A.U = u;
            A.coefs2 = w;
            launch_deriv<DM_HVP>(A, b.hvp, ws, s);
        } else if (w) {   // w_t grad m_t only: the reverse mode of eval with coefficients w
            A.coefs = w;
            launch_deriv<DM_DX>(A, b.dx, ws, s);
        } else {
            clear_u64((unsigned long long *)ggX, N * n, s);
        }
    }
    if (ggY && N > 0) {
        DerivArgs A = deriv_args(f, enc, X, N, ggY);
        A.U = u;
        A.coefs2 = w;
        launch_deriv<DM_DIRD>(A, b.dird, ws, s);
    }
    if (ggC && T > 0) {
        if (N == 0 || !u) {
            clear_u64((unsigned long long *)ggC, T, s);
        } else {
            uint64_t *senc = at<uint64_t>(ws, b.senc);
            double *part = at<double>(ws, b.part);
            hipLaunchKernelGGL(k_encode_support, dim3(grid1(T, 256)), dim3(256), 0, s, f->exps, T, n, senc,
                               (const int64_t *)nullptr);
            const size_t lds = 2 * (size_t)b.cp * n * sizeof(double);
            hipLaunchKernelGGL(k_backward2_dc, dim3(grid1(T, BWC_THREADS), (unsigned)b.nchunks), dim3(BWC_THREADS),
                               lds, s, f->row_ptr, P, f->exps, n, T, X, u, N, gY, part, (const uint64_t *)senc, b.cp);
            hipLaunchKernelGGL(k_backward_dc_reduce, dim3(grid1(T, 256)), dim3(256), 0, s, (const double *)part, T,
                               b.nchunks, ggC);
        }
    }
    LAUNCH_CHECK();
    return POLY_OK;
}

// --------------------------------------------------------------- plans
//
// A plan is the pipeline simplify -> jacobian -> gradient values of a
// polynomial matrix, recorded once into a HIP graph.  Every size that the
// eager entry points read back (the simplified term counts, the Jacobian's
// term counts) stays on the device: the Jacobian is formed over worst-case
// work items and capacities, its factor lists are encoded up to the count
// the device wrote, and evaluation units skip what lies past it.

}  // extern "C"

struct poly_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

struct PipePlan {
    SimplifyPlan sp;
    FormPlan form;
    size_t enc = 0, part = 0, total = 0;
    int64_t jcap = 0, S = 1;
};

PipePlan plan_pipeline(const poly_csr *in, int64_t N)
{
    PipePlan pp;
    const int n = in->nvars;
    const int64_t P = in->npolys, T = total_terms(in);
    pp.sp = plan_simplify(P, T, in->row_ptr_host, n, (uint32_t)in->max_exp + 1);
    Layout L;
    L.off = pp.sp.total;
    pp.jcap = grad_terms_bound(T, n);
    pp.form = plan_form_bound(P, T, n, L);
    pp.enc = L.take(16 * std::max<int64_t>(pp.jcap, 1));
    pp.S = eval_segments(P * n, N, pp.jcap);
    pp.part = L.take(eval_partial_bytes(P * n, N, pp.S));
    pp.total = L.total();
    return pp;
}

poly_status check_pipeline(const poly_csr *in, const double *X, int64_t N, const poly_csr *simp,
                           const poly_csr *jac, const double *G)
{
    poly_status st = check_csr(in, true);
    if (st != POLY_OK) return st;
    if (N < 0) return POLY_ERR_ARG;
    if (!simp && !jac && !G) return POLY_OK;   // workspace query
    if ((st = check_csr(simp, false)) != POLY_OK) return st;
    if ((st = check_csr(jac, false)) != POLY_OK) return st;
    const int n = in->nvars;
    const int64_t P = in->npolys, T = total_terms(in);
    if (simp->nvars != n || simp->npolys != P || simp->capacity < T || simp->max_exp < in->max_exp) return POLY_ERR_ARG;
    if (jac->nvars != n || jac->npolys != P * n || jac->capacity < grad_terms_bound(T, n)) return POLY_ERR_ARG;
    if (P > 0 && N > 0 && (!X || !G)) return POLY_ERR_ARG;
    return POLY_OK;
}

}  // namespace

extern "C" {

poly_status poly_plan_workspace(const poly_csr *in, int64_t N, size_t *ws_bytes)
{
    poly_status st = check_pipeline(in, nullptr, N, nullptr, nullptr, nullptr);
    if (st != POLY_OK) return st;
    if (!ws_bytes) return POLY_ERR_ARG;
    const PipePlan pp = plan_pipeline(in, N);
    if (!pp.sp.ok) return POLY_ERR_UNSUPPORTED;
    *ws_bytes = pp.total;
    return POLY_OK;
}

poly_status poly_plan_create(const poly_csr *in, double zero_tol, const double *X, int64_t N, poly_csr *simplified,
                             poly_csr *jac, double *G, void *ws, size_t ws_bytes, void *stream, poly_plan **plan)
{
    if (!plan) return POLY_ERR_ARG;
    *plan = nullptr;
    poly_status st = check_pipeline(in, X, N, simplified, jac, G);
    if (st != POLY_OK) return st;
    if (!(zero_tol >= 0.0)) return POLY_ERR_ARG;
    if (!stream) return POLY_ERR_ARG;   // the legacy null stream cannot be captured
    const PipePlan pp = plan_pipeline(in, N);
    if (!pp.sp.ok) return POLY_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < pp.total) return POLY_ERR_WORKSPACE;
    const int n = in->nvars;
    const int64_t P = in->npolys;
    hipStream_t s = (hipStream_t)stream;
    ensure_lds_attrs();
    (void)device_cus();
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return POLY_ERR_HIP;
    int32_t *status = at<int32_t>(ws, 0);
    clear_u64(at<unsigned long long>(ws, 0), 1, s);
    if (P == 0) {
        clear_u64((unsigned long long *)simplified->row_ptr, 1, s);
        clear_u64((unsigned long long *)jac->row_ptr, 1, s);
    } else {
        st = run_simplify(in, simplified, zero_tol, ws, pp.sp, s);
        if (st == POLY_OK) {
            FormArgs F = form_args(simplified->row_ptr, simplified->exps, simplified->coefs, n, 0, 0, status,
                                   (int32_t)POLY_ERR_CAPACITY);
            F.out_rp = jac->row_ptr;
            F.out_exps = jac->exps;
            F.out_coefs = jac->coefs;
            F.capacity = jac->capacity;
            run_form(pp.form, F, ws, s);
            if (N > 0) {
                uint32_t *enc = at<uint32_t>(ws, pp.enc);
                hipLaunchKernelGGL(k_encode_factors, dim3(grid1(pp.jcap, 256)), dim3(256), 0, s, jac->exps, pp.jcap, n,
                                   enc, (const int64_t *)(jac->row_ptr + P * n), ws_maxdeg(ws));
                EvalArgs A;
                memset(&A, 0, sizeof(A));
                A.maxdeg = ws_maxdeg(ws);
                A.rp = jac->row_ptr;
                A.exps = jac->exps;
                A.coefs = jac->coefs;
                A.n = n;
                A.X = X;
                A.N = N;
                A.Q = P * n;
                A.mode = OUT_GRAD;
                A.Y = G;
                A.term_limit = pp.jcap;
                launch_eval_blocks(A, enc, at<double>(ws, pp.part), pp.S, s);
            }
        }
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (st != POLY_OK || ec != hipSuccess || hipGetLastError() != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != POLY_OK ? st : POLY_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return POLY_ERR_HIP;
    }
    poly_plan *p = new (std::nothrow) poly_plan;
    if (!p) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return POLY_ERR_HIP;
    }
    p->graph = graph;
    p->exec = exec;
    *plan = p;
    return POLY_OK;
}

poly_status poly_plan_launch(const poly_plan *plan, void *stream)
{
    if (!plan || !plan->exec) return POLY_ERR_ARG;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? POLY_OK : POLY_ERR_HIP;
}

poly_status poly_plan_destroy(poly_plan *plan)
{
    if (!plan) return POLY_OK;
    poly_status st = POLY_OK;
    if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) st = POLY_ERR_HIP;
    if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) st = POLY_ERR_HIP;
    delete plan;
    return st;
}

// ----------------------------------------------------------- dense (shared set)

poly_status poly_eval_dense_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec, int32_t nslices,
                                      size_t *ws_bytes)
{
    return dense_workspace(n, K, P, N, prec, nslices, ws_bytes);
}

poly_status poly_eval_dense(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P,
                            const double *C, int64_t N, const double *X, double *Y, poly_prec prec,
                            int32_t nslices, void *ws, size_t ws_bytes, void *stream)
{
    return dense_run(n, K, basis, max_exp, P, C, N, X, Y, prec, nslices, ws, ws_bytes, (hipStream_t)stream, 1);
}

poly_status poly_eval_dense_backward_workspace(int32_t n, int64_t K, int64_t P, int64_t N, poly_prec prec,
                                               int32_t nslices, size_t *ws_bytes)
{
    return dense_bwd_workspace(n, K, P, N, prec, nslices, ws_bytes);
}

poly_status poly_eval_dense_backward(int32_t n, int64_t K, const uint8_t *basis, int32_t max_exp, int64_t P,
                                     const double *C, int64_t N, const double *X, const double *gY, double *dC,
                                     double *dX, poly_prec prec, int32_t nslices, void *ws, size_t ws_bytes,
                                     void *stream)
{
    return dense_bwd_run(n, K, basis, max_exp, P, C, N, X, gY, dC, dX, prec, nslices, ws, ws_bytes,
                         (hipStream_t)stream);
}

}  // extern "C"
