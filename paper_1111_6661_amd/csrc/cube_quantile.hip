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

#include "cube_quantile_plan.h"
#include "cube_scan.h"

namespace cube {

// Reads of the box made by the calling thread's last successful
// cube_quantiles call.
thread_local int g_quant_reads = 0;

namespace {

constexpr int Q_THREADS = 1024;
constexpr int Q_MAX_RANKS = 2 * CUBE_MAX_QUANTILES;   // index + 1 fits a byte
constexpr size_t Q_LDS = 160 * 1024 - 256;  // dynamic LDS of one block, static aside
constexpr int Q_ACC = 32768;                // slots << bin width never exceeds this
constexpr size_t Q_TAB = QP_TAB_MAX;        // bytes: T1, T2, T3 at most

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
    Claim claim;                   // the partition (its counter zero on entry)
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
        if (NL == 0) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const float v = x[j];
                const bool ok = v == v;
                valid += (unsigned int)__popcll(__builtin_amdgcn_ballot_w64(ok));
                // one histogram, blanks skipped (they are rare)
                if (ok) atomicAdd(&lds[((order_key(v) >> 20) << clog) + cbase], 1u);
            }
        } else {
            // Histogram row g of each voxel: 0 (no wanted prefix) counts
            // nothing.  The tables are read level by level for all NV voxels
            // before any count is added: the counts live in the same LDS, so
            // a table read after an add could not be moved ahead of it, and
            // the voxels' lookups would run one after another.  With two or
            // three table levels the key fields are single bit-field extracts
            // (the one-level pass measured slower with them: 2.52 against
            // 2.34 ms on the brick).
            unsigned int k[NV], g[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                k[j] = order_key(x[j]);
                g[j] = t1[k[j] >> 20];
            }
            if (NL >= 2) {
#pragma unroll
                for (int j = 0; j < NV; ++j)
                    g[j] = t2[(g[j] << w2) | __builtin_amdgcn_ubfe(k[j], 20 - w2, w2)];
            }
            if (NL >= 3) {
#pragma unroll
                for (int j = 0; j < NV; ++j)
                    g[j] = t3[(g[j] << w3) | __builtin_amdgcn_ubfe(k[j], 20 - w2 - w3, w3)];
            }
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const unsigned int idx =
                    (g[j] << wb) | (NL >= 2 ? __builtin_amdgcn_ubfe(k[j], shift, wb)
                                            : (k[j] >> shift) & bmask);
                if (x[j] == x[j] && g[j] != 0u) atomicAdd(&lds[(idx << clog) + cbase], 1u);
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
    scan_box(a.g, st, a.claim);
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
    unsigned long long *acc = nullptr;    // Q_ACC counters, the valid counter, the chunk counter
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
        if ((e = hipMalloc(&w.acc, (Q_ACC + 2) * 8)) != hipSuccess ||
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
int quant_pass(QuantWorkspace *w, const Box &box, const Geom &g, int nl, int shift, int width,
               int w2, int w3, int slots, int t2_bytes, int t3_bytes)
{
    hipError_t e;
    const size_t n = (size_t)slots << width;          // counters read back
    const size_t hist = (size_t)(nl == 0 ? 1 : slots + 1) << width; // LDS words per copy
    const size_t tab = nl == 0 ? 0 : 4096 + (nl >= 2 ? t2_bytes : 0) + (nl >= 3 ? t3_bytes : 0);
    if (n > (size_t)Q_ACC || slots > Q_MAX_RANKS || tab > Q_TAB || hist * 4 + tab > Q_LDS)
        return fail(CUBE_EINVAL, "quantile pass too large");
    if ((e = hipMemsetAsync(w->acc, 0, (Q_ACC + 2) * 8, nullptr)) != hipSuccess)
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
    int blocks = 0, chunks = 0;
    const int rc = scan_plan(box, k, Q_THREADS, lds, &blocks, &chunks);
    if (rc) return rc;
    a.claim.ctr = (unsigned int *)(w->acc + Q_ACC + 1);
    a.claim.nc = chunks;
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

// The passes on the GPU for the host-side plan (cube_quantile_plan.h).
struct GpuPasses {
    QuantWorkspace *w;
    Box box;
    Geom g;
    int reads = 0;  // reads of the box so far
    int first(const unsigned long long **counts, unsigned long long *n)
    {
        ++reads;
        const int rc = quant_pass(w, box, g, 0, 20, 12, 0, 0, 1, 0, 0);
        if (rc) return rc;
        *counts = w->h_acc;
        *n = w->h_acc[Q_ACC];
        return CUBE_OK;
    }
    // The tables are already staged in w->h_tab, which quant_pass uploads.
    int refine(const QuantPassSpec &s, const unsigned char *, const unsigned long long **counts)
    {
        ++reads;
        const int rc = quant_pass(w, box, g, s.nl, s.shift, s.width, s.w2, s.w3, s.slots,
                                  s.t2_bytes, s.t3_bytes);
        if (rc) return rc;
        *counts = w->h_acc;
        return CUBE_OK;
    }
};

int run_quantiles(const Box &box, const double *q, int m, double *out, uint64_t *n_valid_out)
{
    QuantWorkspace *w = nullptr;
    int rc = quant_ws(&w);
    if (rc) return rc;
    GpuPasses P;
    P.w = w;
    P.box = box;
    // Work units for the static grid (two blocks per CU) and for every chunk
    // of a dynamic partition (scan_plan's automatic or set chunk size).
    const int cl = scan_chunk_log2(box);
    const long long units = cl ? chunks_of(box.n, cl) : 0;
    const long long grid = (long long)cu_count() * 2;
    scan_geom(box, units > grid ? units : grid, &P.g);
    rc = quantiles_run(P, q, m, out, n_valid_out, w->h_tab, 1);
    if (rc == 1) return fail(CUBE_EINVAL, "no valid voxel");
    if (rc == CUBE_OK) g_quant_reads = P.reads;
    return rc;
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
    CUBE_GUARD_BEGIN
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
    CUBE_GUARD_END
}

int cube_last_quantile_reads(void) { return g_quant_reads; }

}  // extern "C"
