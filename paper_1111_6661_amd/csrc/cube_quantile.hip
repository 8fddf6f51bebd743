// cube_quantile.hip -- exact quantiles of the valid voxels: every wanted
// rank is refined side by side, so that any number of levels costs three or
// four reads of the cube.  The median and quantiles are the paper's example
// of a global, multi-pass task (Section 3).
//
// Each wanted rank is found in the 32-bit order key of the voxels (the key
// orders like the value, -0 before +0) a few bits at a time, as in
// cube_select.hip, but every pass keeps one histogram per distinct key
// prefix still in play, side by side in LDS:
//   pass 0: one 4096-bin histogram of the top 12 key bits;
//   then, when the ranks fall in at most 8 distinct top buckets and number
//   at most 96, 12 and 8 more bits (up to 8 histograms of 4096 bins, then
//   up to 96 of 256);
//   otherwise 8, 6 and 6 more bits (up to 128 histograms of 256 bins, then
//   128 of 64, then 128 of 64).
// A voxel finds its histogram through a chain of direct-mapped LDS byte
// tables, one per level of the prefix.  Entries hold index + 1 (0: none),
// and row 0 of every further table is all zero, so a voxel outside the
// wanted prefixes falls through to 0 with no test: the table of the top 12
// key bits gives its index among the wanted 12-bit prefixes, each further
// table, indexed by that entry and the level's next key bits, its index
// among the longer prefixes.  Only voxels that end at a wanted prefix count
// (histogram row 0 is laid out but never written).  No search.  The
// host reads each pass's counts back (at most 256 KB) and builds the next
// pass's tables.  A level q takes the voxels of ranks j = floor(q (n - 1))
// and j + 1 and interpolates between them in FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "cube_scan.h"

namespace cube {

namespace {

constexpr int Q_THREADS = 1024;
constexpr int Q_MAX_RANKS = 2 * CUBE_MAX_QUANTILES;   // index + 1 fits a byte
constexpr size_t Q_LDS = 160 * 1024 - 256;  // dynamic LDS of one block, static aside
constexpr int Q_ACC = 32768;                // slots << bin width never exceeds this
constexpr size_t Q_TAB = 4096 + 9 * 4096 + 129 * 64;  // bytes: T1, T2, T3 at most

struct QuantArgs {
    Geom g;
    int32_t shift, width;          // this pass bins key bits [shift, shift + width)
    int32_t w2, w3;                // bits of the second and third prefix levels
    int32_t slots;                 // histograms (prefixes) in this pass
    int32_t copies_log2;           // LDS copies of each histogram
    int32_t t2_bytes, t3_bytes;    // sizes of the second and third tables
    const unsigned char *tab;      // T1 (4096 bytes), T2, T3, back to back
    unsigned long long *acc;       // slots << width counters, zero on entry
    unsigned long long *n_valid;   // pass 0: valid voxels, zero on entry
};

// NL: prefix levels of this pass (0 for the first pass).
template <int NL>
struct QuantStep {
    unsigned int *lds;
    const unsigned char *t1, *t2, *t3;
    int shift, w2, w3, clog, cbase;
    unsigned int bmask;
    int wb;
    unsigned int valid;            // first pass: valid voxels seen by this wavefront

    template <int NV>
    __device__ __forceinline__ void operator()(const float (&x)[NV])
    {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const float v = x[j];
            const bool ok = v == v;
            if (NL == 0) valid += (unsigned int)__popcll(__builtin_amdgcn_ballot_w64(ok));
            const unsigned int k = order_key(v);
            if (NL == 0) {
                // one histogram, blanks skipped (they are rare)
                if (ok) atomicAdd(&lds[((k >> 20) << clog) + cbase], 1u);
            } else {
                // histogram row g: 0 (no wanted prefix) counts nothing
                unsigned int g = t1[k >> 20];
                if (NL >= 2) g = t2[(g << w2) | ((k >> (20 - w2)) & ((1u << w2) - 1u))];
                if (NL >= 3) g = t3[(g << w3) | ((k >> (20 - w2 - w3)) & ((1u << w3) - 1u))];
                const unsigned int idx = (g << wb) | ((k >> shift) & bmask);
                if (ok && g != 0u) atomicAdd(&lds[(idx << clog) + cbase], 1u);
            }
        }
    }
};

template <int NL>
__global__ void __launch_bounds__(Q_THREADS) k_quant(QuantArgs a)
{
    extern __shared__ unsigned int lds[];
    __shared__ unsigned int s_valid;
    const int tid = threadIdx.x, B = blockDim.x;
    const int nbins = 1 << a.width;
    const int rows = NL == 0 ? 1 : a.slots + 1;   // after the first pass, row 0 is unused
    const int words = (rows * nbins) << a.copies_log2;
    for (int i = tid; i < words; i += B) lds[i] = 0u;
    // The tables follow the histograms in LDS (all sizes are multiples of 4).
    unsigned int *tw = lds + words;
    const int tab_words = NL == 0 ? 0 : (4096 + (NL >= 2 ? a.t2_bytes : 0) +
                                         (NL >= 3 ? a.t3_bytes : 0)) / 4;
    const unsigned int *src = (const unsigned int *)a.tab;
    for (int i = tid; i < tab_words; i += B) tw[i] = src[i];
    if (tid == 0) s_valid = 0u;
    __syncthreads();

    QuantStep<NL> st;
    st.lds = lds;
    st.t1 = (const unsigned char *)tw;
    st.t2 = st.t1 + 4096;
    st.t3 = st.t2 + a.t2_bytes;
    st.shift = a.shift;
    st.w2 = a.w2;
    st.w3 = a.w3;
    st.wb = a.width;
    st.bmask = (unsigned int)nbins - 1u;
    st.clog = a.copies_log2;
    st.cbase = tid & 63 & ((1 << a.copies_log2) - 1);
    st.valid = 0u;
    scan_box(a.g, st);
    // Every lane of a wavefront holds the same count (sums of ballots).
    if (NL == 0 && (tid & 63) == 0 && st.valid) atomicAdd(&s_valid, st.valid);
    __syncthreads();
    // Flush the histograms (after the first pass, rows 1..: row 0 is
    // never written).
    const int C = 1 << a.copies_log2;
    const int first = NL == 0 ? 0 : nbins;
    for (int b = tid; b < a.slots * nbins; b += B) {
        unsigned int sum = 0;
        for (int c = 0; c < C; ++c) sum += lds[((b + first) << a.copies_log2) + c];
        if (sum) atomicAdd(&a.acc[b], (unsigned long long)sum);
    }
    if (NL == 0 && tid == 0 && s_valid) atomicAdd(a.n_valid, (unsigned long long)s_valid);
}

struct QuantWorkspace {
    unsigned long long *acc = nullptr;    // Q_ACC counters + 1 valid counter
    unsigned char *tab = nullptr;         // the prefix tables
    unsigned long long *h_acc = nullptr;  // pinned copy of the counters
    unsigned char *h_tab = nullptr;       // pinned staging of the tables
};

std::mutex g_qmu;
QuantWorkspace g_qws[64];
bool g_qws_ready[64];

int quant_ws(QuantWorkspace **out)
{
    int dev = 0;
    hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return fail(CUBE_EINVAL, "device index out of range");
    if (!g_qws_ready[dev]) {
        QuantWorkspace &w = g_qws[dev];
        hipError_t e;
        if ((e = hipMalloc(&w.acc, (Q_ACC + 1) * 8)) != hipSuccess ||
            (e = hipMalloc(&w.tab, Q_TAB)) != hipSuccess ||
            (e = hipHostMalloc(&w.h_acc, (Q_ACC + 1) * 8)) != hipSuccess ||
            (e = hipHostMalloc(&w.h_tab, Q_TAB)) != hipSuccess)
            return hip_fail(e, "quantile workspace");
        g_qws_ready[dev] = true;
    }
    *out = &g_qws[dev];
    return CUBE_OK;
}

// One pass: zero the counters, upload the tables (already staged in h_tab),
// launch, read the counters back (slots << width of them, and the valid
// count after the first pass).  All on the null stream; returns after the
// copy.  nl: prefix levels (0 for the first pass); w2, w3 their widths.
int quant_pass(QuantWorkspace *w, const Geom &g, int blocks, int nl, int shift, int width,
               int w2, int w3, int slots, int t2_bytes, int t3_bytes)
{
    hipError_t e;
    const size_t n = (size_t)slots << width;          // counters read back
    const size_t hist = (size_t)(nl == 0 ? 1 : slots + 1) << width; // LDS words per copy
    const size_t tab = nl == 0 ? 0 : 4096 + (nl >= 2 ? t2_bytes : 0) + (nl >= 3 ? t3_bytes : 0);
    if (n > (size_t)Q_ACC || slots > Q_MAX_RANKS || tab > Q_TAB || hist * 4 + tab > Q_LDS)
        return fail(CUBE_EINVAL, "quantile pass too large");
    if ((e = hipMemsetAsync(w->acc, 0, (Q_ACC + 1) * 8, nullptr)) != hipSuccess)
        return hip_fail(e, "quantile counters");
    if (tab &&
        (e = hipMemcpyAsync(w->tab, w->h_tab, tab, hipMemcpyHostToDevice, nullptr)) != hipSuccess)
        return hip_fail(e, "quantile tables");
    // Up to eight copies of each histogram, as many as fit beside the tables.
    int clog = 0;
    while (clog < 3 && (hist << (clog + 1)) * 4 + tab <= Q_LDS) ++clog;
    const size_t lds = (hist << clog) * 4 + tab;
    QuantArgs a;
    memset(&a, 0, sizeof a);
    a.g = g;
    a.shift = shift;
    a.width = width;
    a.w2 = w2;
    a.w3 = w3;
    a.slots = slots;
    a.copies_log2 = clog;
    a.t2_bytes = t2_bytes;
    a.t3_bytes = t3_bytes;
    a.tab = w->tab;
    a.acc = w->acc;
    a.n_valid = w->acc + Q_ACC;
    const void *k = nl == 0   ? reinterpret_cast<const void *>(&k_quant<0>)
                    : nl == 1 ? reinterpret_cast<const void *>(&k_quant<1>)
                    : nl == 2 ? reinterpret_cast<const void *>(&k_quant<2>)
                              : reinterpret_cast<const void *>(&k_quant<3>);
    if (lds > 64 * 1024 &&
        (e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
            hipSuccess)
        return hip_fail(e, "quantile LDS");
    void *args[] = {&a};
    if ((e = hipLaunchKernel(k, dim3((unsigned)blocks), dim3(Q_THREADS), args, lds, nullptr)) !=
        hipSuccess)
        return hip_fail(e, "quantile launch");
    if ((e = hipMemcpyAsync(w->h_acc, w->acc, n * 8, hipMemcpyDeviceToHost, nullptr)) !=
            hipSuccess ||
        (nl == 0 && (e = hipMemcpyAsync(w->h_acc + Q_ACC, w->acc + Q_ACC, 8,
                                        hipMemcpyDeviceToHost, nullptr)) != hipSuccess) ||
        (e = hipStreamSynchronize(nullptr)) != hipSuccess)
        return hip_fail(e, "quantile counts");
    return CUBE_OK;
}

// A rank being refined: the key bits found so far (at the top of `key`) and
// the rank left inside that prefix.
struct Want {
    unsigned long long rank;
    unsigned int key;
};

// The bin of `h` (nbins counters) holding rank r; r becomes the rank
// inside that bin.  The counts sum to more than r by construction.
unsigned int pick_bin(const unsigned long long *h, int nbins, unsigned long long &r)
{
    int b = 0;
    while (b < nbins - 1 && h[b] <= r) r -= h[b++];
    return (unsigned int)b;
}

float key_to_float(unsigned int k)
{
    const unsigned int u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

double interpolate(double a, double b, double f)
{
    if (a == b) return a;
    if (isinf(a) && isinf(b)) return NAN;
    if (isinf(a)) return a;
    if (isinf(b)) return b;
    return a + f * (b - a);
}

// The distinct values of the top `bits` key bits among the wanted ranks,
// ascending.
std::vector<unsigned int> prefixes(const std::vector<Want> &want, int bits)
{
    std::vector<unsigned int> p;
    for (const Want &x : want) p.push_back(x.key >> (32 - bits));
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
    return p;
}

size_t index_of(const std::vector<unsigned int> &p, unsigned int v)
{
    return std::lower_bound(p.begin(), p.end(), v) - p.begin();
}

size_t index_of_rank(const std::vector<unsigned long long> &r, unsigned long long v)
{
    return std::lower_bound(r.begin(), r.end(), v) - r.begin();
}

int run_quantiles(const Box &box, const double *q, int m, double *out, uint64_t *n_valid_out)
{
    QuantWorkspace *w = nullptr;
    int rc = quant_ws(&w);
    if (rc) return rc;
    const int blocks = cu_count() * 2;
    Geom g;
    scan_geom(box, blocks, &g);

    // The top 12 bits, and the valid count.
    if ((rc = quant_pass(w, g, blocks, 0, 20, 12, 0, 0, 1, 0, 0))) return rc;
    const unsigned long long n = w->h_acc[Q_ACC];
    if (n_valid_out) *n_valid_out = n;
    if (n == 0) return fail(CUBE_EINVAL, "no valid voxel");

    // The ranks the levels need, ascending and distinct (at most 2m).
    std::vector<unsigned long long> ranks;
    for (int i = 0; i < m; ++i) {
        const double h = q[i] * (double)(n - 1);
        const double j = floor(h);
        ranks.push_back((unsigned long long)j);
        if (h - j > 0.0) ranks.push_back((unsigned long long)j + 1);
    }
    std::sort(ranks.begin(), ranks.end());
    ranks.erase(std::unique(ranks.begin(), ranks.end()), ranks.end());
    std::vector<Want> want(ranks.size());
    for (size_t i = 0; i < ranks.size(); ++i) {
        want[i].rank = ranks[i];
        want[i].key = pick_bin(w->h_acc, 4096, want[i].rank) << 20;
    }

    // The remaining 20 bits: 12 + 8 when the ranks lie in at most 8 top
    // buckets and number at most 96 (the tables and histograms of both
    // passes fit in LDS), else 8 + 6 + 6.
    const bool wide = prefixes(want, 12).size() <= 8 && want.size() <= 96;
    static const int wide_w[] = {12, 8}, narrow_w[] = {8, 6, 6};
    const int *widths = wide ? wide_w : narrow_w;
    const int npass = wide ? 2 : 3;
    int lev[3] = {12, 0, 0};  // widths of the prefix levels
    int done = 12;            // key bits found so far
    for (int p = 0; p < npass; ++p) {
        const int nl = p + 1;  // prefix levels of this pass
        const int width = widths[p];
        // Level tables, entries index + 1 (0: none): T1 maps the top 12
        // bits to the index among the 12-bit prefixes; T2 maps (that entry,
        // the next lev[1] bits) to the index among the longer prefixes, with
        // row 0 all zero; T3 likewise one level further.
        unsigned char *t1 = w->h_tab;
        memset(t1, 0, 4096);
        const std::vector<unsigned int> p1 = prefixes(want, 12);
        for (size_t i = 0; i < p1.size(); ++i) t1[p1[i]] = (unsigned char)(i + 1);
        std::vector<unsigned int> deepest = p1;
        int t2_bytes = 0, t3_bytes = 0;
        if (nl >= 2) {
            const std::vector<unsigned int> p2 = prefixes(want, 12 + lev[1]);
            unsigned char *t2 = t1 + 4096;
            t2_bytes = (int)((p1.size() + 1) << lev[1]);
            memset(t2, 0, (size_t)t2_bytes);
            for (size_t i = 0; i < p2.size(); ++i) {
                const unsigned int up = (unsigned int)index_of(p1, p2[i] >> lev[1]) + 1;
                t2[(up << lev[1]) | (p2[i] & ((1u << lev[1]) - 1u))] = (unsigned char)(i + 1);
            }
            if (nl >= 3) {
                const std::vector<unsigned int> p3 = prefixes(want, 12 + lev[1] + lev[2]);
                unsigned char *t3 = t2 + t2_bytes;
                t3_bytes = (int)((p2.size() + 1) << lev[2]);
                memset(t3, 0, (size_t)t3_bytes);
                for (size_t i = 0; i < p3.size(); ++i) {
                    const unsigned int up = (unsigned int)index_of(p2, p3[i] >> lev[2]) + 1;
                    t3[(up << lev[2]) | (p3[i] & ((1u << lev[2]) - 1u))] = (unsigned char)(i + 1);
                }
                deepest = p3;
            } else {
                deepest = p2;
            }
        }
        const int shift = 32 - done - width;
        if ((rc = quant_pass(w, g, blocks, nl, shift, width, lev[1], lev[2], (int)deepest.size(),
                             t2_bytes, t3_bytes)))
            return rc;
        for (Want &x : want) {
            const size_t slot = index_of(deepest, x.key >> (32 - done));
            const unsigned int b =
                pick_bin(w->h_acc + (slot << width), 1 << width, x.rank);
            x.key |= b << shift;
        }
        if (nl < 3) lev[nl] = width;
        done += width;
    }

    // The levels: the voxels of ranks j and j + 1, interpolated.
    auto value_of = [&](unsigned long long r) {
        return (double)key_to_float(want[index_of_rank(ranks, r)].key);
    };
    for (int i = 0; i < m; ++i) {
        const double h = q[i] * (double)(n - 1);
        const double j = floor(h);
        const double f = h - j;
        const double a = value_of((unsigned long long)j);
        const double b = f > 0.0 ? value_of((unsigned long long)j + 1) : a;
        out[i] = interpolate(a, b, f);
    }
    return CUBE_OK;
}

}  // namespace

void quant_release()
{
    std::lock_guard<std::mutex> lk(g_qmu);
    for (int d = 0; d < 64; ++d) {
        if (!g_qws_ready[d]) continue;
        QuantWorkspace &w = g_qws[d];
        hipFree(w.acc);
        hipFree(w.tab);
        hipHostFree(w.h_acc);
        hipHostFree(w.h_tab);
        w = QuantWorkspace();
        g_qws_ready[d] = false;
    }
}

}  // namespace cube

using namespace cube;

extern "C" {

int cube_quantiles(const float *ptr, const int64_t *dims, const double *q, int32_t m,
                   double *out, uint64_t *n_valid)
{
    if (!q || !out) return fail(CUBE_EINVAL, "q or out is NULL");
    if (m < 1 || m > CUBE_MAX_QUANTILES)
        return fail(CUBE_EINVAL, "m=%d outside [1, %d]", m, CUBE_MAX_QUANTILES);
    for (int i = 0; i < m; ++i)
        if (!(q[i] >= 0.0 && q[i] <= 1.0))
            return fail(CUBE_EINVAL, "level q[%d] outside [0, 1]", i);
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (!rc) rc = check_box_device(&b);
    if (rc) return rc;
    if (b.n == 0) {
        if (n_valid) *n_valid = 0;
        return fail(CUBE_EINVAL, "empty box");
    }
    std::lock_guard<std::mutex> lk(g_qmu);
    return run_quantiles(b, q, m, out, n_valid);
}

}  // extern "C"
