// cube_quantile.hip -- exact quantiles of the valid voxels: several ranks
// refined side by side, so that any number of levels costs the same three
// reads of the cube as one (up to eight distinct leading key buckets; more
// add one read per eight).  The median and quantiles are the paper's example
// of a global, multi-pass task (Section 3).
//
// Each wanted rank is found in the 32-bit order key of the voxels (the key
// orders like the value, -0 before +0) 12, 12 and 8 bits at a time, as in
// cube_select.hip.  Here every pass keeps one histogram per distinct key
// prefix still in play, side by side in LDS:
//   pass 0: one 4096-bin histogram of the top 12 key bits;
//   pass 1: for up to 8 distinct top-12 buckets, a 4096-bin histogram each
//           of the next 12 bits (a 4096-entry LDS table maps a voxel's top
//           bits to its histogram, or to none);
//   pass 2: for up to 128 distinct 24-bit prefixes, a 256-bin histogram each
//           of the last 8 bits (the table, then a short list per top bucket).
// The host reads each pass's counts back (a few hundred KB at most) and
// chooses the next pass's prefixes.  A level q takes the voxels of ranks
// j = floor(q (n - 1)) and j + 1 and interpolates between them in FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "cube_scan.h"

namespace cube {

namespace {

constexpr int Q_THREADS = 1024;
constexpr int Q_MAX_SLOTS1 = 8;          // pass-1 histograms per read
constexpr int Q_MAX_SLOTS2 = 2 * CUBE_MAX_QUANTILES;
constexpr size_t Q_LDS_HIST = 128 * 1024;
constexpr int Q_ACC = 32768;             // max(8 * 4096, 128 * 256) counters

struct QuantArgs {
    Geom g;
    int32_t pass;
    int32_t nbins;                 // bins per histogram: 4096 or 256
    int32_t slots;                 // histograms in this pass
    int32_t copies_log2;           // LDS copies of each histogram
    int32_t slots1;                // pass 2: top buckets in the table
    const short *top;              // passes 1, 2: top-12 bucket -> slot (-1: none)
    const unsigned short *off;     // pass 2: slot1 s -> mids [off[s], off[s + 1])
    const unsigned short *mids;    // pass 2: middle 12 bits of each 24-bit prefix
    unsigned long long *acc;       // slots * nbins counters, zero on entry
    unsigned long long *n_valid;   // pass 0: valid voxels, zero on entry
};

template <int PASS>
struct QuantStep {
    unsigned int *lds;
    const short *top;
    const unsigned short *off, *mids;
    int clog, cbase;
    unsigned int valid;            // pass 0: valid voxels seen by this wavefront

    template <int NV>
    __device__ __forceinline__ void operator()(const float (&x)[NV])
    {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const float v = x[j];
            const bool ok = v == v;
            if (PASS == 0) valid += (unsigned int)__popcll(__builtin_amdgcn_ballot_w64(ok));
            const unsigned int k = order_key(v);
            int idx = -1;
            if (ok) {
                if (PASS == 0) {
                    idx = (int)(k >> 20);
                } else if (PASS == 1) {
                    const int s = top[k >> 20];
                    if (s >= 0) idx = (s << 12) | (int)((k >> 8) & 0xfffu);
                } else {
                    const int s = top[k >> 20];
                    if (s >= 0) {
                        const unsigned short mid = (unsigned short)((k >> 8) & 0xfffu);
                        for (int t = off[s]; t < off[s + 1]; ++t)
                            if (mids[t] == mid) idx = (t << 8) | (int)(k & 0xffu);
                    }
                }
            }
            if (idx >= 0) atomicAdd(&lds[(idx << clog) + cbase], 1u);
        }
    }
};

template <int PASS>
__global__ void __launch_bounds__(Q_THREADS) k_quant(QuantArgs a)
{
    extern __shared__ unsigned int lds[];
    __shared__ short s_top[4096];
    __shared__ unsigned short s_off[Q_MAX_SLOTS2 + 1], s_mids[Q_MAX_SLOTS2];
    __shared__ unsigned int s_valid;
    const int tid = threadIdx.x, B = blockDim.x;
    const int words = (a.slots * a.nbins) << a.copies_log2;
    for (int i = tid; i < words; i += B) lds[i] = 0u;
    if (PASS > 0)
        for (int i = tid; i < 4096; i += B) s_top[i] = a.top[i];
    if (PASS == 2) {
        for (int i = tid; i <= a.slots1; i += B) s_off[i] = a.off[i];
        for (int i = tid; i < a.slots; i += B) s_mids[i] = a.mids[i];
    }
    if (tid == 0) s_valid = 0u;
    __syncthreads();

    QuantStep<PASS> st;
    st.lds = lds;
    st.top = s_top;
    st.off = s_off;
    st.mids = s_mids;
    st.clog = a.copies_log2;
    st.cbase = tid & 63 & ((1 << a.copies_log2) - 1);
    st.valid = 0u;
    scan_box(a.g, st);
    // Every lane of a wavefront holds the same count (sums of ballots).
    if (PASS == 0 && (tid & 63) == 0 && st.valid) atomicAdd(&s_valid, st.valid);
    __syncthreads();
    const int C = 1 << a.copies_log2;
    for (int b = tid; b < a.slots * a.nbins; b += B) {
        unsigned int sum = 0;
        for (int c = 0; c < C; ++c) sum += lds[(b << a.copies_log2) + c];
        if (sum) atomicAdd(&a.acc[b], (unsigned long long)sum);
    }
    if (PASS == 0 && tid == 0 && s_valid) atomicAdd(a.n_valid, (unsigned long long)s_valid);
}

struct QuantWorkspace {
    unsigned long long *acc = nullptr;    // Q_ACC counters + 1 valid counter
    short *tab = nullptr;                 // top table, offsets, mids
    unsigned long long *h_acc = nullptr;  // pinned copy of the counters
    short *h_tab = nullptr;               // pinned staging of the tables
};

constexpr size_t TAB_TOP = 4096, TAB_OFF = Q_MAX_SLOTS2 + 1, TAB_MIDS = Q_MAX_SLOTS2;
constexpr size_t TAB_WORDS = TAB_TOP + TAB_OFF + TAB_MIDS;

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
// back (slots * nbins of them, and the valid count after pass 0).  All on
// the null stream; returns after the copy.
int quant_pass(QuantWorkspace *w, const Geom &g, int blocks, int pass, int nbins, int slots,
               size_t tab_words, int slots1 = 0)
{
    hipError_t e;
    const size_t n = (size_t)slots * nbins;
    if ((e = hipMemsetAsync(w->acc, 0, (Q_ACC + 1) * 8, nullptr)) != hipSuccess)
        return hip_fail(e, "quantile counters");
    if (tab_words &&
        (e = hipMemcpyAsync(w->tab, w->h_tab, tab_words * 2, hipMemcpyHostToDevice, nullptr)) !=
            hipSuccess)
        return hip_fail(e, "quantile tables");
    int clog = 0;
    while (clog < 3 && (n << (clog + 1)) * 4 <= Q_LDS_HIST) ++clog;
    const size_t lds = (n << clog) * 4;
    QuantArgs a;
    memset(&a, 0, sizeof a);
    a.g = g;
    a.pass = pass;
    a.nbins = nbins;
    a.slots = slots;
    a.copies_log2 = clog;
    a.slots1 = slots1;
    a.top = w->tab;
    a.off = (const unsigned short *)(w->tab + TAB_TOP);
    a.mids = (const unsigned short *)(w->tab + TAB_TOP + TAB_OFF);
    a.acc = w->acc;
    a.n_valid = w->acc + Q_ACC;
    const void *k = pass == 0   ? reinterpret_cast<const void *>(&k_quant<0>)
                    : pass == 1 ? reinterpret_cast<const void *>(&k_quant<1>)
                                : reinterpret_cast<const void *>(&k_quant<2>);
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
        (pass == 0 && (e = hipMemcpyAsync(w->h_acc + Q_ACC, w->acc + Q_ACC, 8,
                                          hipMemcpyDeviceToHost, nullptr)) != hipSuccess) ||
        (e = hipStreamSynchronize(nullptr)) != hipSuccess)
        return hip_fail(e, "quantile counts");
    return CUBE_OK;
}

// A rank being refined: the key bits found so far and the rank left inside
// the current prefix.
struct Want {
    unsigned long long rank;
    unsigned int b0, b1, b2;
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

    // Pass 0: the top 12 bits, and the valid count.
    if ((rc = quant_pass(w, g, blocks, 0, 4096, 1, 0))) return rc;
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
        want[i].b0 = pick_bin(w->h_acc, 4096, want[i].rank);
    }

    // Pass 1, eight top buckets per read: the middle 12 bits.
    std::vector<unsigned int> tops;
    for (const Want &x : want) tops.push_back(x.b0);
    std::sort(tops.begin(), tops.end());
    tops.erase(std::unique(tops.begin(), tops.end()), tops.end());
    for (size_t r0 = 0; r0 < tops.size(); r0 += Q_MAX_SLOTS1) {
        const int ns = (int)std::min(tops.size() - r0, (size_t)Q_MAX_SLOTS1);
        for (size_t i = 0; i < TAB_TOP; ++i) w->h_tab[i] = -1;
        for (int s = 0; s < ns; ++s) w->h_tab[tops[r0 + s]] = (short)s;
        if ((rc = quant_pass(w, g, blocks, 1, 4096, ns, TAB_TOP))) return rc;
        for (Want &x : want)
            for (int s = 0; s < ns; ++s)
                if (x.b0 == tops[r0 + s]) x.b1 = pick_bin(w->h_acc + (size_t)s * 4096, 4096, x.rank);
    }

    // Pass 2: the last 8 bits under each distinct 24-bit prefix, grouped by
    // top bucket (slot1 = the bucket's index in `tops`).
    std::vector<unsigned int> pre;
    for (const Want &x : want) pre.push_back((x.b0 << 12) | x.b1);
    std::sort(pre.begin(), pre.end());
    pre.erase(std::unique(pre.begin(), pre.end()), pre.end());
    for (size_t i = 0; i < TAB_TOP; ++i) w->h_tab[i] = -1;
    unsigned short *off = (unsigned short *)(w->h_tab + TAB_TOP);
    unsigned short *mids = (unsigned short *)(w->h_tab + TAB_TOP + TAB_OFF);
    size_t t = 0;
    for (size_t s = 0; s < tops.size(); ++s) {
        w->h_tab[tops[s]] = (short)s;
        off[s] = (unsigned short)t;
        while (t < pre.size() && (pre[t] >> 12) == tops[s]) {
            mids[t] = (unsigned short)(pre[t] & 0xfffu);
            ++t;
        }
    }
    off[tops.size()] = (unsigned short)t;
    if ((rc = quant_pass(w, g, blocks, 2, 256, (int)pre.size(), TAB_WORDS, (int)tops.size())))
        return rc;
    for (Want &x : want) {
        const size_t slot = std::lower_bound(pre.begin(), pre.end(), (x.b0 << 12) | x.b1) -
                            pre.begin();
        x.b2 = pick_bin(w->h_acc + slot * 256, 256, x.rank);
    }

    // The levels: the voxels of ranks j and j + 1, interpolated.
    auto value_of = [&](unsigned long long r) {
        const size_t i = std::lower_bound(ranks.begin(), ranks.end(), r) - ranks.begin();
        return (double)key_to_float((want[i].b0 << 20) | (want[i].b1 << 8) | want[i].b2);
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
