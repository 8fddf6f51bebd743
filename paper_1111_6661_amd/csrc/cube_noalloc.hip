// cube_noalloc.hip -- the allocation-free form of the fused single-box pass.
//
// cube_stats_hist_noalloc runs the same kernel as cube_stats_hist_async, but
// its scratch memory (the wavefront records of the local stage, the
// last-block ticket and the global histogram accumulators) is one
// file-scope device array instead of a per-stream workspace, so a call
// makes no device or host allocation.  Every call on a device shares that
// device's copy of the array: calls that overlap on one device race.
#include <string.h>

#include <mutex>

#include "cube_internal.h"

namespace cube {

namespace {

constexpr size_t NA_RECS = CUBE_NOALLOC_MAX_RECORDS;
constexpr size_t NA_REC_BYTES = NA_RECS * sizeof(WaveRec);
constexpr size_t NA_TICKET_BYTES = 256;
constexpr size_t NA_ACC_WORDS = (size_t)CUBE_MAX_BINS + 3;
constexpr size_t NA_BYTES = NA_REC_BYTES + NA_TICKET_BYTES + NA_ACC_WORDS * 8;
static_assert(NA_REC_BYTES % 256 == 0, "records end on a 256-byte boundary");

// The scratch array.  In host code its name is a host-side stand-in: only
// the address hipGetSymbolAddress returns for a device is used.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[NA_MAX_DEVICES];  // per device; null until set up

// Set-up on the current device, once: the device address of its scratch
// array, and the device facts the planner caches (CU count), so that later
// calls touch no allocating code.
int scratch_of_current(int *dev_out, unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NA_MAX_DEVICES)
        return fail(CUBE_EINVAL, "device %d beyond the %d the allocation-free call supports", dev,
                    NA_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        (void)cu_count();
        g_na_ptr[dev] = (unsigned char *)p;
    }
    *dev_out = dev;
    *out = g_na_ptr[dev];
    return CUBE_OK;
}

// Zero the ticket and the first `acc_words` accumulators (a fill kernel, so
// the call stays valid under stream capture).
__global__ void k_na_clear(unsigned int *ticket, unsigned long long *acc, int acc_words)
{
    if (blockIdx.x == 0 && threadIdx.x < NA_TICKET_BYTES / 4) ticket[threadIdx.x] = 0u;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < acc_words;
         i += gridDim.x * blockDim.x)
        acc[i] = 0ull;
}

}  // namespace

}  // namespace cube

using namespace cube;

extern "C" int cube_stats_hist_noalloc(const float *ptr, const int64_t *dims, float lo, float hi,
                                       int32_t nbins, cube_stats_t *dev_out,
                                       uint64_t *dev_counts, void *stream)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    if (!dev_out) return fail(CUBE_EINVAL, "stats output is NULL");
    if (!dev_counts) return fail(CUBE_EINVAL, "counts output is NULL");
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (rc) return rc;
    HistRange range;
    if ((rc = check_range(lo, hi, nbins, &range))) return rc;
    int dev = 0;
    unsigned char *base = nullptr;
    if ((rc = scratch_of_current(&dev, &base))) return rc;
    if ((rc = check_box_device(&b))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (b.n == 0) return write_empty(dev_out, (unsigned long long *)dev_counts, nbins, s);

    Plan p;
    if ((rc = make_plan(b, true, 1, nbins, &p))) return rc;
    const long long waves = p.threads / 64;
    if (p.chunks > 0) {
        // A dynamic partition keeps one record per chunk: at most NA_RECS
        // chunks (each block still flushes its LDS counters in time).
        if (p.chunks > (int)NA_RECS) {
            p.chunks = (int)NA_RECS;
            if (p.blocks > p.chunks) p.blocks = p.chunks;
            cut_rows(p.g, p.chunks);
        }
    } else if ((long long)p.blocks * waves > (long long)NA_RECS) {
        int t = 0, bl = 0, c = 0, u = 0;
        get_launch(&t, &bl, &c, &u);
        if (bl != 0)
            return fail(CUBE_EINVAL,
                        "launch shape of %d blocks x %d threads needs %lld wave records; the "
                        "allocation-free scratch holds %zu",
                        p.blocks, p.threads, (long long)p.blocks * waves, NA_RECS);
        // An automatic or tuned grid is narrowed to the records the scratch
        // holds; every block must still cover under 2^31 voxels.
        p.blocks = (int)(NA_RECS / waves);
        if ((long long)(b.n >> 31) + 1 > p.blocks)
            return fail(CUBE_EINVAL, "box of %llu voxels too large for the allocation-free scratch",
                        (unsigned long long)b.n);
        cut_rows(p.g, p.blocks);
    }

    WaveRec *recs = (WaveRec *)base;
    unsigned int *ticket = (unsigned int *)(base + NA_REC_BYTES);
    unsigned long long *acc = (unsigned long long *)(base + NA_REC_BYTES + NA_TICKET_BYTES);
    hipLaunchKernelGGL(k_na_clear, dim3((unsigned)((nbins + 255) / 256)), dim3(256), 0, s,
                       ticket, acc, nbins);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scratch clear launch");

    PassArgs a;
    memset(&a, 0, sizeof a);
    a.g = p.g;
    a.nbins = nbins;
    a.copies_log2 = p.copies_log2;
    a.range = range;
    a.recs = recs;
    a.ticket = ticket;
    a.hist_acc = acc;
    a.out = dev_out;
    a.counts = (unsigned long long *)dev_counts;
    a.accum_mode = accum_mode();
    a.n_chunks = p.chunks;
    e = launch_pass(a, true, p.hist, p.threads, p.blocks, p.lds, p.unroll, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return CUBE_OK;
    CUBE_GUARD_END
}
