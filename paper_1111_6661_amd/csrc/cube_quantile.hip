// cube_quantile.hip -- exact quantiles of the valid voxels: every wanted
// rank is refined side by side, so that any number of levels costs three or
// four reads of the cube.  The median and quantiles are the paper's example
// of a global, multi-pass task (Section 3).
//
// Each wanted rank is found in the 32-bit order key of the voxels (the key
// orders like the value, -0 before +0) a few bits at a time, as in
// cube_select.hip, but every pass keeps one histogram per distinct key
// prefix still in play, side by side in LDS (at most 128 KB):
//   pass 0: one 4096-bin histogram of the top 12 key bits;
//   then, when the ranks fall in at most 8 distinct top buckets, 12 and 8
//   more bits (up to 8 histograms of 4096 bins, then up to 128 of 256);
//   otherwise 8, 8 and 4 more bits (up to 128 histograms of 256 bins, then
//   128 of 256, then 128 of 16).
// A voxel finds its histogram through a 4096-entry LDS table indexed by its
// top 12 key bits: in the pass after the first the table gives the
// histogram itself; later it gives the group of prefixes under that bucket,
// which the voxel scans for its own (groups are short: the prefixes of the
// wanted ranks under one 12-bit bucket).  The host reads each pass's
// counts back (at most 256 KB) and chooses the next pass's prefixes.  A
// level q takes the voxels of ranks j = floor(q (n - 1)) and j + 1 and
// interpolates between them in FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "cube_scan.h"

namespace cube {

namespace {

constexpr int Q_THREADS = 1024;
constexpr int Q_MAX_SLOTS = 2 * CUBE_MAX_QUANTILES;   // distinct prefixes per pass
constexpr size_t Q_LDS_HIST = 128 * 1024;
constexpr int Q_ACC = 32768;             // slots * bins never exceeds this

struct QuantArgs {
    Geom g;
    int32_t shift, width;          // this pass bins key bits [shift, shift + width)
    int32_t slots;                 // histograms (prefixes) in this pass
    int32_t groups;                // top-12 buckets among the prefixes
    int32_t copies_log2;           // LDS copies of each histogram
    const short *top;              // top-12 bucket -> group (-1: none)
    const unsigned short *off;     // group g -> prefixes [off[g], off[g + 1])
    const unsigned int *pre;       // the prefixes (key >> (shift + width)), ascending
    unsigned long long *acc;       // slots << width counters, zero on entry
    unsigned long long *n_valid;   // pass 0: valid voxels, zero on entry
};

// Pass modes: the first pass (no prefix), a pass whose prefixes are the top
// 12 bits (the table gives the histogram), a pass with longer prefixes.
enum { Q_FIRST = 0, Q_DIRECT = 1, Q_SCAN = 2 };

template <int MODE>
struct QuantStep {
    unsigned int *lds;
    const short *top;
    const unsigned short *off;
    const unsigned int *pre;
    int shift, pshift, clog, cbase;
    unsigned int bmask;
    unsigned int valid;            // first pass: valid voxels seen by this wavefront

    template <int NV>
    __device__ __forceinline__ void operator()(const float (&x)[NV])
    {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const float v = x[j];
            const bool ok = v == v;
            if (MODE == Q_FIRST)
                valid += (unsigned int)__popcll(__builtin_amdgcn_ballot_w64(ok));
            const unsigned int k = order_key(v);
            int idx = -1;
            if (ok) {
                if (MODE == Q_FIRST) {
                    idx = (int)(k >> 20);
                } else {
                    const int g = top[k >> 20];
                    if (MODE == Q_DIRECT) {
                        if (g >= 0)
                            idx = (int)(((unsigned int)g << (pshift - shift)) |
                                        ((k >> shift) & bmask));
                    } else if (g >= 0) {
                        const unsigned int p = k >> pshift;
                        for (int t = off[g]; t < off[g + 1]; ++t)
                            if (pre[t] == p)
                                idx = (int)(((unsigned int)t << (pshift - shift)) |
                                            ((k >> shift) & bmask));
                    }
                }
            }
            if (idx >= 0) atomicAdd(&lds[(idx << clog) + cbase], 1u);
        }
    }
};

template <int MODE>
__global__ void __launch_bounds__(Q_THREADS) k_quant(QuantArgs a)
{
    extern __shared__ unsigned int lds[];
    __shared__ short s_top[4096];
    __shared__ unsigned short s_off[Q_MAX_SLOTS + 1];
    __shared__ unsigned int s_pre[Q_MAX_SLOTS];
    __shared__ unsigned int s_valid;
    const int tid = threadIdx.x, B = blockDim.x;
    const int nbins = 1 << a.width;
    const int words = (a.slots * nbins) << a.copies_log2;
    for (int i = tid; i < words; i += B) lds[i] = 0u;
    if (MODE != Q_FIRST) {
        for (int i = tid; i < 4096; i += B) s_top[i] = a.top[i];
        for (int i = tid; i <= a.groups; i += B) s_off[i] = a.off[i];
        for (int i = tid; i < a.slots; i += B) s_pre[i] = a.pre[i];
    }
    if (tid == 0) s_valid = 0u;
    __syncthreads();

    QuantStep<MODE> st;
    st.lds = lds;
    st.top = s_top;
    st.off = s_off;
    st.pre = s_pre;
    st.shift = a.shift;
    st.pshift = a.shift + a.width;
    st.bmask = (unsigned int)nbins - 1u;
    st.clog = a.copies_log2;
    st.cbase = tid & 63 & ((1 << a.copies_log2) - 1);
    st.valid = 0u;
    scan_box(a.g, st);
    // Every lane of a wavefront holds the same count (sums of ballots).
    if (MODE == Q_FIRST && (tid & 63) == 0 && st.valid) atomicAdd(&s_valid, st.valid);
    __syncthreads();
    const int C = 1 << a.copies_log2;
    for (int b = tid; b < a.slots * nbins; b += B) {
        unsigned int sum = 0;
        for (int c = 0; c < C; ++c) sum += lds[(b << a.copies_log2) + c];
        if (sum) atomicAdd(&a.acc[b], (unsigned long long)sum);
    }
    if (MODE == Q_FIRST && tid == 0 && s_valid)
        atomicAdd(a.n_valid, (unsigned long long)s_valid);
}

struct QuantWorkspace {
    unsigned long long *acc = nullptr;    // Q_ACC counters + 1 valid counter
    short *tab = nullptr;                 // top table, offsets, mids
    unsigned long long *h_acc = nullptr;  // pinned copy of the counters
    short *h_tab = nullptr;               // pinned staging of the tables
};

// Table layout (16-bit words): top[4096], off[Q_MAX_SLOTS + 1] (padded to an
// even count), then pre[Q_MAX_SLOTS] as 32-bit words.
constexpr size_t TAB_TOP = 4096, TAB_OFF = (Q_MAX_SLOTS + 2) & ~(size_t)1;
constexpr size_t TAB_WORDS = TAB_TOP + TAB_OFF + 2 * Q_MAX_SLOTS;

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
            (e = hipMalloc(&w.tab, TAB_WORDS * 2)) != hipSuccess ||
            (e = hipHostMalloc(&w.h_acc, (Q_ACC + 1) * 8)) != hipSuccess ||
            (e = hipHostMalloc(&w.h_tab, TAB_WORDS * 2)) != hipSuccess)
            return hip_fail(e, "quantile workspace");
        g_qws_ready[dev] = true;
    }
    *out = &g_qws[dev];
    return CUBE_OK;
}

// One pass: zero the counters, upload the tables, launch, read the counters
// back (slots << width of them, and the valid count after the first pass).
// All on the null stream; returns after the copy.
int quant_pass(QuantWorkspace *w, const Geom &g, int blocks, bool first, int shift, int width,
               int slots, int groups)
{
    hipError_t e;
    const size_t n = (size_t)slots << width;
    if (n > (size_t)Q_ACC || slots > Q_MAX_SLOTS || groups > Q_MAX_SLOTS)
        return fail(CUBE_EINVAL, "quantile pass too large");
    if ((e = hipMemsetAsync(w->acc, 0, (Q_ACC + 1) * 8, nullptr)) != hipSuccess)
        return hip_fail(e, "quantile counters");
    if (!first &&
        (e = hipMemcpyAsync(w->tab, w->h_tab, TAB_WORDS * 2, hipMemcpyHostToDevice, nullptr)) !=
            hipSuccess)
        return hip_fail(e, "quantile tables");
    int clog = 0;
    while (clog < 3 && (n << (clog + 1)) * 4 <= Q_LDS_HIST) ++clog;
    const size_t lds = (n << clog) * 4;
    QuantArgs a;
    memset(&a, 0, sizeof a);
    a.g = g;
    a.shift = shift;
    a.width = width;
    a.slots = slots;
    a.groups = groups;
    a.copies_log2 = clog;
    a.top = w->tab;
    a.off = (const unsigned short *)(w->tab + TAB_TOP);
    a.pre = (const unsigned int *)(w->tab + TAB_TOP + TAB_OFF);
    a.acc = w->acc;
    a.n_valid = w->acc + Q_ACC;
    // Prefixes of exactly the top 12 bits: the table gives the histogram.
    const void *k = first                 ? reinterpret_cast<const void *>(&k_quant<Q_FIRST>)
                    : shift + width == 20 ? reinterpret_cast<const void *>(&k_quant<Q_DIRECT>)
                                          : reinterpret_cast<const void *>(&k_quant<Q_SCAN>);
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
        (first && (e = hipMemcpyAsync(w->h_acc + Q_ACC, w->acc + Q_ACC, 8,
                                      hipMemcpyDeviceToHost, nullptr)) != hipSuccess) ||
        (e = hipStreamSynchronize(nullptr)) != hipSuccess)
        return hip_fail(e, "quantile counts");
    return CUBE_OK;
}

// A rank being refined: the key bits found so far (the prefix) and the
// rank left inside that prefix.
struct Want {
    unsigned long long rank;
    unsigned int prefix;
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

int run_quantiles(const Box &box, const double *q, int m, double *out, uint64_t *n_valid_out)
{
    QuantWorkspace *w = nullptr;
    int rc = quant_ws(&w);
    if (rc) return rc;
    const int blocks = cu_count() * 2;
    Geom g;
    scan_geom(box, blocks, &g);

    // The top 12 bits, and the valid count.
    if ((rc = quant_pass(w, g, blocks, true, 20, 12, 1, 0))) return rc;
    const unsigned long long n = w->h_acc[Q_ACC];
    if (n_valid_out) *n_valid_out = n;
    if (n == 0) return fail(CUBE_EINVAL, "no valid voxel");

    // The ranks the levels need, ascending and distinct.
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
        want[i].prefix = pick_bin(w->h_acc, 4096, want[i].rank);
    }

    // The remaining 20 bits: 12 + 8 when the ranks lie in at most 8 top
    // buckets (a 4096-bin histogram per bucket fits), else 8 + 8 + 4.
    std::vector<unsigned int> pre;
    auto distinct = [&]() {
        pre.clear();
        for (const Want &x : want) pre.push_back(x.prefix);
        std::sort(pre.begin(), pre.end());
        pre.erase(std::unique(pre.begin(), pre.end()), pre.end());
    };
    distinct();
    static const int wide[] = {12, 8}, narrow[] = {8, 8, 4};
    const int *widths = pre.size() <= 8 ? wide : narrow;
    const int npass = pre.size() <= 8 ? 2 : 3;
    int done = 12;  // key bits found so far
    for (int p = 0; p < npass; ++p) {
        if (p) distinct();
        const int width = widths[p];
        const int shift = 32 - done - width;
        // Tables: prefixes ascending, grouped by their top 12 bits.
        short *top = w->h_tab;
        unsigned short *off = (unsigned short *)(w->h_tab + TAB_TOP);
        unsigned int *pv = (unsigned int *)(w->h_tab + TAB_TOP + TAB_OFF);
        for (size_t i = 0; i < TAB_TOP; ++i) top[i] = -1;
        int groups = 0;
        for (size_t t = 0; t < pre.size(); ++t) {
            const unsigned int t12 = pre[t] >> (done - 12);
            if (t == 0 || t12 != (pre[t - 1] >> (done - 12))) {
                top[t12] = (short)groups;
                off[groups++] = (unsigned short)t;
            }
            pv[t] = pre[t];
        }
        off[groups] = (unsigned short)pre.size();
        if ((rc = quant_pass(w, g, blocks, false, shift, width, (int)pre.size(), groups)))
            return rc;
        for (Want &x : want) {
            const size_t slot = std::lower_bound(pre.begin(), pre.end(), x.prefix) - pre.begin();
            const unsigned int b = pick_bin(w->h_acc + (slot << width), 1 << width, x.rank);
            x.prefix = (x.prefix << width) | b;
        }
        done += width;
    }

    // The levels: the voxels of ranks j and j + 1, interpolated.
    auto value_of = [&](unsigned long long r) {
        const size_t i = std::lower_bound(ranks.begin(), ranks.end(), r) - ranks.begin();
        return (double)key_to_float(want[i].prefix);
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
