// cube_capi.hip -- the C ABI of the cube statistics library: argument
// validation, launch planning, per-stream workspaces and result copies.
// Declarations and the contract of every entry point are in cubestats.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "cube_internal.h"

namespace cube {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(CUBE_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

std::vector<uint64_t> fault_inject(const char *kind)
{
    std::vector<uint64_t> out;
    const char *env = getenv("CUBE_FAULT_INJECT");
    if (!env) return out;
    const size_t klen = strlen(kind);
    bool match = false;
    for (const char *p = env; *p;) {
        const char *end = strchr(p, ',');
        const size_t len = end ? (size_t)(end - p) : strlen(p);
        const char *colon = (const char *)memchr(p, ':', len);
        const char *num = p;
        if (colon) {
            match = (size_t)(colon - p) == klen && strncmp(p, kind, klen) == 0;
            num = colon + 1;
        }
        char *stop = nullptr;
        const unsigned long long v = strtoull(num, &stop, 10);
        if (match && stop != num && stop == p + len) out.push_back((uint64_t)v);
        if (!end) break;
        p = end + 1;
    }
    return out;
}

// The precision mode and the launch-shape override belong to the calling
// thread: a call never takes a setting another thread made (the server's
// worker, for one, always runs with the defaults).
thread_local int g_accum = CUBE_ACCUM_FP64MERGE;

int accum_mode() { return g_accum; }

thread_local int g_threads = 0, g_blocks = 0, g_copies = 0, g_unroll = 0;
thread_local int g_hot = -1;

void set_hot_override(int hot) { g_hot = hot; }
int hot_override() { return g_hot; }
thread_local int g_chunk = -1;  // partition override: -1 none, 0 static, k chunks of 2^k
void set_chunk_override(int chunk_log2) { g_chunk = chunk_log2; }
int chunk_override() { return g_chunk; }

void get_launch(int *threads, int *blocks, int *copies, int *unroll)
{
    *threads = g_threads;
    *blocks = g_blocks;
    *copies = g_copies;
    *unroll = g_unroll;
}

constexpr int MAX_BLOCKS = 4096;
constexpr int MAX_WAVES_PER_BLOCK = 16;
constexpr size_t REC_CAP = (size_t)MAX_BLOCKS * MAX_WAVES_PER_BLOCK;
constexpr size_t LDS_BUDGET = 132 * 1024;  // one 1024-thread histogram block per CU

// One workspace per (device, stream): partial records, the ticket, the
// histogram accumulators (kept at zero between launches by the kernel) and
// the result staging buffers.
struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    WaveRec *recs = nullptr;
    unsigned int *ticket = nullptr;
    unsigned long long *hist_acc = nullptr;
    cube_stats_t *d_out = nullptr;
    unsigned long long *d_counts = nullptr;
    HistRange *d_range = nullptr;
    cube_stats_t *h_out = nullptr;        // pinned
    unsigned long long *h_counts = nullptr;
    hipEvent_t used = nullptr;            // recorded after the last work queued with it
    std::mutex mu;                        // held by synchronous calls
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;
std::map<int, int> g_cus;

// Waits for the last work queued with the workspace through its event, not
// through its stream: the caller may have destroyed that stream already.
void free_ws(Workspace *w)
{
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(w->device);
    if (w->used) {
        hipEventSynchronize(w->used);
        hipEventDestroy(w->used);
    }
    hipFree(w->recs);
    hipFree(w->ticket);
    hipFree(w->hist_acc);
    hipFree(w->d_out);
    hipFree(w->d_counts);
    hipFree(w->d_range);
    hipHostFree(w->h_out);
    hipHostFree(w->h_counts);
    hipSetDevice(prev);
    delete w;
}

int get_ws(hipStream_t s, Workspace **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return CUBE_OK;
    }
    Workspace *w = new Workspace;
    w->device = dev;
    w->stream = s;
    const size_t nacc = (size_t)CUBE_MAX_BINS + 3;
    bool ok = hipEventCreateWithFlags(&w->used, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&w->recs, REC_CAP * sizeof(WaveRec)) == hipSuccess &&
              hipMalloc(&w->ticket, 256) == hipSuccess &&
              hipMalloc(&w->hist_acc, nacc * 8) == hipSuccess &&
              hipMalloc(&w->d_out, sizeof(cube_stats_t)) == hipSuccess &&
              hipMalloc(&w->d_counts, nacc * 8) == hipSuccess &&
              hipMalloc(&w->d_range, 256) == hipSuccess &&
              hipHostMalloc(&w->h_out, sizeof(cube_stats_t)) == hipSuccess &&
              hipHostMalloc(&w->h_counts, nacc * 8) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        free_ws(w);
        return fail(CUBE_ENOMEM, "workspace allocation failed");
    }
    if ((e = hipMemset(w->ticket, 0, 256)) != hipSuccess ||
        (e = hipMemset(w->hist_acc, 0, nacc * 8)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
        free_ws(w);
        return hip_fail(e, "workspace initialisation");
    }
    g_ws[key] = w;
    *out = w;
    return CUBE_OK;
}

// Record that work using `w` was queued on `s` (after a successful enqueue).
int mark_ws(Workspace *w, hipStream_t s)
{
    const hipError_t e = hipEventRecord(w->used, s);
    return e == hipSuccess ? CUBE_OK : hip_fail(e, "workspace event");
}

int stream_counter(hipStream_t s, unsigned int **ctr)
{
    Workspace *w = nullptr;
    const int rc = get_ws(s, &w);
    if (rc) return rc;
    *ctr = w->ticket + CHUNK_CTR_WORD;
    return CUBE_OK;
}

int stream_used(hipStream_t s)
{
    Workspace *w = nullptr;
    const int rc = get_ws(s, &w);
    return rc ? rc : mark_ws(w, s);
}

// Free the workspaces of stream `s` (one per device it was used on; a live
// stream handle names one stream process-wide).
void release_ws(hipStream_t s)
{
    std::vector<Workspace *> gone;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto it = g_ws.begin(); it != g_ws.end();) {
            if (it->first.second == s) {
                gone.push_back(it->second);
                it = g_ws.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (Workspace *w : gone) free_ws(w);
}

int cu_count()
{
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cus.find(dev);
    if (it != g_cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
        n = 256;
    g_cus[dev] = n;
    return n;
}

// ---------------------------------------------------------------- validation

// One past the last voxel of a non-empty box, in floats from its first:
// (nz-1)*sz + (ny-1)*sy + nx, with every product and sum checked.  False
// when it does not fit in 2^62 floats, so that neither it nor its size in
// bytes can wrap around (a wrapped extent would let a box reaching far past
// its allocation pass the bounds check, and the kernel would fault).
static bool box_end_floats(const Box &b, uint64_t *end)
{
    const uint64_t sy = b.ny > 1 ? (uint64_t)b.sy : 0, sz = b.nz > 1 ? (uint64_t)b.sz : 0;
    uint64_t ey = 0, ez = 0, e = 0;
    if (__builtin_mul_overflow((uint64_t)(b.ny - 1), sy, &ey) ||
        __builtin_mul_overflow((uint64_t)(b.nz - 1), sz, &ez) ||
        __builtin_add_overflow(ey, ez, &e) || __builtin_add_overflow(e, (uint64_t)b.nx, &e) ||
        e > ((uint64_t)1 << 62))
        return false;
    *end = e;
    return true;
}

int check_box(const float *ptr, const int64_t *dims, Box *b)
{
    if (!dims) return fail(CUBE_EINVAL, "dims is NULL");
    b->ptr = ptr;
    b->nx = dims[0];
    b->ny = dims[1];
    b->nz = dims[2];
    if (b->nx < 0 || b->ny < 0 || b->nz < 0)
        return fail(CUBE_EINVAL, "negative extent (%lld, %lld, %lld)", (long long)b->nx,
                    (long long)b->ny, (long long)b->nz);
    b->sy = dims[3] == 0 ? b->nx : dims[3];
    b->sz = dims[4];
    if (b->nx == 0 || b->ny == 0 || b->nz == 0) {
        b->n = 0;
        // nothing is read; the dense plane pitch only if it is representable
        if (b->sz == 0 && __builtin_mul_overflow(b->sy, b->ny, &b->sz)) b->sz = 0;
        return CUBE_OK;
    }
    if (b->nx > (int64_t)1 << 40 || b->ny > (int64_t)1 << 40 || b->nz > (int64_t)1 << 40)
        return fail(CUBE_EINVAL, "extent too large");
    if (b->ny > 1 && b->sy < b->nx)
        return fail(CUBE_EINVAL, "row pitch sy=%lld < nx=%lld", (long long)b->sy,
                    (long long)b->nx);
    // The plane's own extent, (ny-1)*sy + nx, checked (sy >= nx >= 1 here
    // when ny > 1), then the dense plane pitch sy*ny when sz is 0.
    int64_t plane = b->nx, dense = b->sy;
    if (b->ny > 1 && (__builtin_mul_overflow(b->sy, b->ny - 1, &plane) ||
                      __builtin_add_overflow(plane, b->nx, &plane) ||
                      __builtin_mul_overflow(b->sy, b->ny, &dense)))
        return fail(CUBE_EINVAL, "row pitch sy=%lld too large", (long long)b->sy);
    if (b->sz == 0) b->sz = dense;
    if (b->nz > 1 && b->sz < plane)
        return fail(CUBE_EINVAL, "plane pitch sz=%lld overlaps the previous plane",
                    (long long)b->sz);
    uint64_t end = 0;
    if (!box_end_floats(*b, &end))
        return fail(CUBE_EINVAL, "box extent overflows (pitches sy=%lld, sz=%lld)",
                    (long long)b->sy, (long long)b->sz);
    b->n = (uint64_t)b->nx * (uint64_t)b->ny * (uint64_t)b->nz;
    if (!ptr) return fail(CUBE_EINVAL, "data pointer is NULL");
    if ((uintptr_t)ptr & 3) return fail(CUBE_EINVAL, "data pointer is not 4-byte aligned");
    return CUBE_OK;
}

// Checks that need the HIP runtime (after check_box succeeded).
int check_box_device(const Box *b)
{
    const float *ptr = b->ptr;
    if (b->n == 0) return CUBE_OK;
    // The pointer must be device memory and the whole box must lie inside
    // its allocation: a read outside it would fault the GPU.
    hipPointerAttribute_t pa;
    hipError_t e = hipPointerGetAttributes(&pa, ptr);
    if (e != hipSuccess) {
        hipGetLastError();
        return fail(CUBE_EINVAL, "data pointer is not GPU memory");
    }
    if (pa.type != hipMemoryTypeDevice && pa.type != hipMemoryTypeManaged)
        return fail(CUBE_EINVAL, "data pointer is not device memory");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess) {
        hipGetLastError();
        return fail(CUBE_EINVAL, "cannot find the allocation of the data pointer");
    }
    uint64_t last = 0;  // one past the last voxel, in floats (checked, < 2^62)
    if (!box_end_floats(*b, &last)) return fail(CUBE_EINVAL, "box extent overflows");
    const uint64_t room = (uint64_t)((uintptr_t)base + size - (uintptr_t)ptr);  // bytes
    if ((uintptr_t)ptr < (uintptr_t)base || last > room / 4u)
        return fail(CUBE_EINVAL, "box extends past the end of its allocation");
    int dev = 0;
    hipGetDevice(&dev);
    if (pa.device != dev)
        return fail(CUBE_EINVAL, "data lives on device %d, current device is %d", pa.device,
                    dev);
    return CUBE_OK;
}

int check_range(float lo, float hi, int32_t nbins, HistRange *r)
{
    if (nbins < 1 || nbins > CUBE_MAX_BINS)
        return fail(CUBE_EINVAL, "nbins=%d outside [1, %d]", nbins, CUBE_MAX_BINS);
    if (isnan(lo) || isnan(hi)) return fail(CUBE_EINVAL, "NaN histogram bound");
    if (isinf(lo) || isinf(hi)) return fail(CUBE_EINVAL, "infinite histogram bound");
    if (hi < lo) return fail(CUBE_EINVAL, "hi < lo");
    volatile float width = hi - lo;  // one FP32 rounding, as the kernels see it
    if (isinf(width)) return fail(CUBE_EINVAL, "hi - lo overflows float32");
    float scale = 0.f;
    if (width != 0.f) {
        volatile float nb = (float)nbins;
        scale = nb / width;
        if (isinf(scale)) return fail(CUBE_EINVAL, "range too narrow for %d bins", nbins);
    }
    r->lo = lo;
    r->hi = hi;
    r->scale = scale;
    r->ok = 1;
    return CUBE_OK;
}

// ------------------------------------------------------------------ planning

void collapse(const Box &b, Geom *g)
{
    int64_t row = b.nx, ny = 1, sy = 0, nz = 1, sz = 0;
    const int64_t n[2] = {b.ny, b.nz}, st[2] = {b.sy, b.sz};
    for (int k = 0; k < 2; ++k) {
        if (n[k] == 1) continue;
        if (ny == 1 && st[k] == row)
            row *= n[k];
        else if (ny == 1) {
            ny = n[k];
            sy = st[k];
        } else if (st[k] == ny * sy)
            ny *= n[k];
        else {
            nz = n[k];
            sz = st[k];
        }
    }
    g->ptr = b.ptr;
    g->row_len = row;
    g->ny = ny;
    g->nz = nz;
    g->sy = sy;
    g->sz = sz;
    g->n_total = b.n;
}

// The partition of a fully automatic launch (no explicit shape, no tuned
// entry): dynamic for large boxes, where blocks on the slower XCDs would
// otherwise set the end of the pass.  Measured with the default shapes on
// dense boxes of 2^25 to 2^31 voxels: chunks of 2^18 voxels beat the static
// partition from 2^27 voxels on for histogram passes (by 1-10 %, growing
// with the box), and chunks of 2^19 from 2^30 on for the statistics pass.
static int default_chunk_log2(bool hist, uint64_t n)
{
    if (hist) return n >= ((uint64_t)1 << 27) ? 18 : 0;
    return n >= ((uint64_t)1 << 30) ? 19 : 0;
}

int make_plan(const Box &b, bool stats, int hist_kind_req, int nbins, Plan *p)
{
    collapse(b, &p->g);
    int threads = g_threads, unroll = g_unroll, copies_req = g_copies;
    long long blocks = g_blocks;
    // With no explicit shape, use the autotuner's choice for this class.
    TunedShape ts;
    const int kind = stats ? (hist_kind_req ? CUBE_Q_FUSED : CUBE_Q_STATS) : CUBE_Q_HIST;
    int hot = 0, chunk_log2 = 0, resident = 0;
    const bool automatic = threads == 0 && unroll == 0 && copies_req == 0 && blocks == 0;
    if (automatic) chunk_log2 = default_chunk_log2(hist_kind_req != 0, b.n);
    if (automatic && tuned_shape(kind, hist_kind_req ? nbins : 1, b.n, &ts)) {
        threads = ts.threads;
        unroll = ts.unroll;
        copies_req = ts.copies;
        blocks = (long long)cu_count() * ts.blocks_per_cu;
        hot = ts.hot;
        chunk_log2 = ts.chunk_log2;
        resident = ts.blocks_per_cu;
    }
    if (g_hot >= 0) hot = g_hot;
    if (g_chunk >= 0) chunk_log2 = g_chunk;
    // Histogram passes over boxes under 2^25 voxels default to 256 threads:
    // their launches are short enough that per-block costs dominate (below).
    const bool small = b.n < ((uint64_t)1 << 25);
    if (threads != 256 && threads != 512 && threads != 1024)
        threads = (hist_kind_req && !small) ? 1024 : 256;
    p->threads = threads;
    p->unroll = (unroll == 2 || unroll == 4) ? unroll : 4;
    p->hist = HIST_NONE;
    p->copies_log2 = 0;
    if (hist_kind_req) {
        if (nbins > 32768) {
            p->hist = HIST_GLOBAL;
        } else {
            p->hist = HIST_LDS;
            int c = copies_req;
            int clog = 0;
            if (c > 0) {
                while ((1 << (clog + 1)) <= c && clog < 5) ++clog;
            } else {
                const size_t words = LDS_BUDGET / 4;
                while (clog < 5 && (size_t)(nbins + 2) << (clog + 1) <= words) ++clog;
            }
            while (clog > 0 && ((size_t)(nbins + 2) << clog) * 4 > 160 * 1024) --clog;
            p->copies_log2 = clog;
            if (hot) p->hist = HIST_HOT;
        }
    }
    p->lds = pass_lds_bytes(stats, p->hist, nbins, p->copies_log2, threads);
    p->chunks = 0;
    if (chunk_log2 > 0 && p->hist != HIST_HOT && accum_mode() == CUBE_ACCUM_FP64MERGE) {
        // Dynamic partition: one persistent wave of blocks (the tuned blocks
        // per CU, else all that fit; an explicit grid as given) claiming
        // chunks of about 2^chunk_log2 voxels.
        // The kernel keeps a ring of wavefront records after its histogram
        // in LDS: fewer histogram copies if both would not fit one block
        // (its static LDS is about 1 KB).
        while (true) {
            p->lds = pass_lds_bytes(stats, p->hist, nbins, p->copies_log2, threads, true);
            if (p->lds + 4096 <= 160 * 1024 || p->hist != HIST_LDS || p->copies_log2 == 0) break;
            --p->copies_log2;
        }
        const int fit = pass_blocks_per_cu(stats, p->hist, threads, p->lds, p->unroll, true);
        const long long chunks = chunks_of(b.n, chunk_log2);
        if (g_blocks == 0) {
            const int per_cu = resident > 0 && resident < fit ? resident : fit;
            blocks = (long long)cu_count() * per_cu;
        }
        if (blocks > chunks) blocks = chunks;
        if (blocks > MAX_BLOCKS) blocks = MAX_BLOCKS;
        if (blocks < 1) blocks = 1;
        p->chunks = (int)chunks;
        p->blocks = (int)blocks;
        cut_rows(p->g, chunks);
        return CUBE_OK;
    }
    const int bpc = pass_blocks_per_cu(stats, p->hist, threads, p->lds, p->unroll);
    // At least four blocks per CU over the launch: with one resident
    // histogram block per CU, four waves of blocks measured faster than one
    // persistent wave on large boxes (shorter per-block ranges, overlapped
    // tails).
    const long long cap = (long long)cu_count() * (bpc < 4 ? 4 : bpc);
    const long long per_block_min = (long long)threads * 16 * 2;  // two main-loop steps
    if (blocks <= 0) {
        blocks = (long long)((b.n + per_block_min - 1) / per_block_min);
        // Every block adds a fixed cost at the end of the pass (its ticket
        // atomic on one address, its release fence, its records for the
        // final merge, and for histograms one flush of every bin; measured
        // at 9-30 ns per block for the first three), while the streaming
        // time falls as n / blocks: the sum is least near sqrt(n) blocks.
        // Measured on boxes of 2^16 to 2^30 voxels, the fastest counts were
        // about sqrt(n) / 16, up to one block per CU for histogram passes
        // (each block flushes its whole LDS histogram) and two for the
        // statistics pass; the largest boxes keep the CU cap (or the tuned
        // shape).
        if (b.n < ((uint64_t)1 << 31)) {
            long long root = (long long)sqrt((double)b.n) / 16;
            const long long mid = (long long)cu_count() * (hist_kind_req ? 1 : 2);
            if (root > mid) root = mid;
            if (blocks > root) blocks = root < 1 ? 1 : root;
        }
        if (blocks > cap) blocks = cap;
    }
    // Per-block LDS counters are 32-bit: keep every block under 2^31 voxels.
    const long long min_blocks = (long long)(b.n >> 31) + 1;
    if (blocks < min_blocks) blocks = min_blocks;
    if (blocks < 1) blocks = 1;
    if (blocks > MAX_BLOCKS) blocks = MAX_BLOCKS;
    if ((size_t)blocks * (threads / 64) > REC_CAP) blocks = (long long)(REC_CAP / (threads / 64));
    p->blocks = (int)blocks;
    cut_rows(p->g, blocks);
    return CUBE_OK;
}

long long chunks_of(uint64_t n, int chunk_log2)
{
    const uint64_t c = (n + ((uint64_t)1 << chunk_log2) - 1) >> chunk_log2;
    if (c < 1) return 1;
    return c > (uint64_t)REC_CAP ? (long long)REC_CAP : (long long)c;
}

void cut_rows(Geom &g, long long blocks)
{
    const long long rows = g.ny * g.nz;
    long long segs = 1;
    if (rows < blocks) segs = (blocks + rows - 1) / rows;
    long long seg_len = (g.row_len + segs - 1) / segs;
    seg_len = (seg_len + 3) & ~3LL;
    if (seg_len < 4) seg_len = 4;
    segs = (g.row_len + seg_len - 1) / seg_len;
    g.seg_len = seg_len;
    g.segs = segs;
    g.n_units = rows * segs;
}

__global__ void k_write_empty(cube_stats_t *out, unsigned long long *counts, int nbins)
{
    const float qn = __int_as_float(0x7fc00000);
    if (out && threadIdx.x == 0) {
        cube_stats_t o;
        o.n_total = o.n_valid = o.n_nan = 0;
        o.min = o.max = qn;
        o.mean = o.m2 = o.std = (double)qn;
        o.flags = CUBE_NO_VALID;
        o.reserved = 0;
        *out = o;
    }
    if (counts)
        for (int i = threadIdx.x; i < nbins + 3; i += blockDim.x) counts[i] = 0ull;
}

int launch(const PassArgs &a, const Plan &p, bool stats, hipStream_t s)
{
    hipError_t e =
        launch_pass(a, stats, p.hist, p.threads, p.blocks, p.lds, p.unroll, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return CUBE_OK;
}

PassArgs base_args(const Workspace *w, const Plan &p, int nbins)
{
    PassArgs a;
    memset(&a, 0, sizeof a);
    a.g = p.g;
    a.nbins = nbins;
    a.copies_log2 = p.copies_log2;
    a.recs = w->recs;
    a.ticket = w->ticket;
    a.hist_acc = w->hist_acc;
    a.accum_mode = g_accum;
    a.n_chunks = p.chunks;
    return a;
}

// The four operations, stream-ordered, with device outputs.
enum Op { OP_STATS, OP_HIST, OP_FUSED, OP_MINMAX };

int run_async(Op op, const float *ptr, const int64_t *dims, float lo, float hi, int32_t nbins,
              cube_stats_t *dev_out, unsigned long long *dev_counts, hipStream_t s,
              Workspace *w)
{
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (rc) return rc;
    if ((rc = check_box_device(&b))) return rc;
    HistRange range = {0.f, 0.f, 0.f, 1};
    if (op == OP_HIST || op == OP_FUSED) {
        if ((rc = check_range(lo, hi, nbins, &range))) return rc;
    } else if (op == OP_MINMAX) {
        if (nbins < 1 || nbins > CUBE_MAX_BINS)
            return fail(CUBE_EINVAL, "nbins=%d outside [1, %d]", nbins, CUBE_MAX_BINS);
    }
    if (op != OP_HIST && !dev_out) return fail(CUBE_EINVAL, "stats output is NULL");
    if (op != OP_STATS && !dev_counts) return fail(CUBE_EINVAL, "counts output is NULL");
    if (b.n == 0) {
        hipLaunchKernelGGL(k_write_empty, dim3(1), dim3(256), 0, s,
                           op == OP_HIST ? nullptr : dev_out,
                           op == OP_STATS ? nullptr : dev_counts, nbins);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? CUBE_OK : hip_fail(e, "empty-box launch");
    }
    Plan p;
    if (op == OP_STATS || op == OP_MINMAX) {
        if ((rc = make_plan(b, true, 0, nbins, &p))) return rc;
        PassArgs a = base_args(w, p, nbins);
        a.out = dev_out;
        if (op == OP_MINMAX) {
            a.want_range = 1;
            a.out_range = w->d_range;
        }
        if ((rc = launch(a, p, true, s))) return rc;
        if (op == OP_STATS) return CUBE_OK;
        Plan p2;
        if ((rc = make_plan(b, false, 1, nbins, &p2))) return rc;
        PassArgs a2 = base_args(w, p2, nbins);
        a2.dev_range = w->d_range;
        a2.counts = dev_counts;
        return launch(a2, p2, false, s);
    }
    const bool stats = op == OP_FUSED;
    if ((rc = make_plan(b, stats, 1, nbins, &p))) return rc;
    PassArgs a = base_args(w, p, nbins);
    a.range = range;
    a.out = dev_out;
    a.counts = dev_counts;
    return launch(a, p, stats, s);
}

int run_pass(const Box &b, bool stats, bool hist, int nbins, const HistRange &range,
             const HistRange *dev_range, cube_stats_t *dev_out, unsigned long long *dev_counts,
             bool accumulate, hipStream_t s)
{
    if (b.n == 0) return fail(CUBE_EINVAL, "run_pass on an empty box");
    Workspace *w = nullptr;
    int rc = get_ws(s, &w);
    if (rc) return rc;
    Plan p;
    if ((rc = make_plan(b, stats, hist ? 1 : 0, nbins, &p))) return rc;
    PassArgs a = base_args(w, p, nbins);
    a.range = range;
    a.dev_range = dev_range;
    a.out = stats ? dev_out : nullptr;
    a.counts = hist ? dev_counts : nullptr;
    a.accumulate = accumulate ? 1 : 0;
    if ((rc = launch(a, p, stats, s))) return rc;
    return mark_ws(w, s);
}

int write_empty(cube_stats_t *dev_out, unsigned long long *dev_counts, int nbins, hipStream_t s)
{
    hipLaunchKernelGGL(k_write_empty, dim3(1), dim3(256), 0, s, dev_out, dev_counts, nbins);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CUBE_OK : hip_fail(e, "empty-box launch");
}

// Argument checks that need no GPU: done before any HIP call.
int precheck(Op op, const float *ptr, const int64_t *dims, float lo, float hi, int32_t nbins)
{
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (rc) return rc;
    HistRange r;
    if (op == OP_HIST || op == OP_FUSED) return check_range(lo, hi, nbins, &r);
    if (op == OP_MINMAX && (nbins < 1 || nbins > CUBE_MAX_BINS))
        return fail(CUBE_EINVAL, "nbins=%d outside [1, %d]", nbins, CUBE_MAX_BINS);
    return CUBE_OK;
}

int run_sync(Op op, const float *ptr, const int64_t *dims, float lo, float hi, int32_t nbins,
             cube_stats_t *out, uint64_t *counts)
{
    if (op != OP_HIST && !out) return fail(CUBE_EINVAL, "stats output is NULL");
    if (op != OP_STATS && !counts) return fail(CUBE_EINVAL, "counts output is NULL");
    int rc = precheck(op, ptr, dims, lo, hi, nbins);
    if (rc) return rc;
    Workspace *w = nullptr;
    rc = get_ws(nullptr, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    rc = run_async(op, ptr, dims, lo, hi, nbins, w->d_out, w->d_counts, nullptr, w);
    if (rc) return rc;
    hipError_t e;
    if (op != OP_HIST &&
        (e = hipMemcpyAsync(w->h_out, w->d_out, sizeof(cube_stats_t), hipMemcpyDeviceToHost,
                            nullptr)) != hipSuccess)
        return hip_fail(e, "result copy");
    if (op != OP_STATS &&
        (e = hipMemcpyAsync(w->h_counts, w->d_counts, ((size_t)nbins + 3) * 8,
                            hipMemcpyDeviceToHost, nullptr)) != hipSuccess)
        return hip_fail(e, "counts copy");
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e, "synchronize");
    if ((rc = mark_ws(w, nullptr))) return rc;
    if (op != OP_HIST) *out = *w->h_out;
    if (op != OP_STATS) memcpy(counts, w->h_counts, ((size_t)nbins + 3) * 8);
    if (op == OP_MINMAX && (w->h_out->flags & CUBE_HIST_BAD_RANGE))
        return fail(CUBE_EINVAL, "the data range [min, max] is not a valid histogram range");
    return CUBE_OK;
}

int run_async_entry(Op op, const float *ptr, const int64_t *dims, float lo, float hi,
                    int32_t nbins, cube_stats_t *dev_out, uint64_t *dev_counts, void *stream)
{
    if (op != OP_HIST && !dev_out) return fail(CUBE_EINVAL, "stats output is NULL");
    if (op != OP_STATS && !dev_counts) return fail(CUBE_EINVAL, "counts output is NULL");
    int rc = precheck(op, ptr, dims, lo, hi, nbins);
    if (rc) return rc;
    Workspace *w = nullptr;
    rc = get_ws((hipStream_t)stream, &w);
    if (rc) return rc;
    rc = run_async(op, ptr, dims, lo, hi, nbins, dev_out, (unsigned long long *)dev_counts,
                   (hipStream_t)stream, w);
    if (rc) return rc;
    return mark_ws(w, (hipStream_t)stream);
}

}  // namespace cube

using namespace cube;

extern "C" {

int cube_abi_version(void) { return CUBE_ABI_VERSION; }

const char *cube_last_error(void) { return g_err.c_str(); }

int cube_stats(const float *ptr, int64_t nx, int64_t ny, int64_t nz, const int64_t *stride,
               cube_stats_t *out)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    const int64_t dims[5] = {nx, ny, nz, stride ? stride[0] : 0, stride ? stride[1] : 0};
    return run_sync(OP_STATS, ptr, dims, 0.f, 0.f, 1, out, nullptr);
    CUBE_GUARD_END
}

int cube_hist(const float *ptr, const int64_t *dims, float lo, float hi, int32_t nbins,
              uint64_t *counts)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_sync(OP_HIST, ptr, dims, lo, hi, nbins, nullptr, counts);
    CUBE_GUARD_END
}

int cube_stats_hist(const float *ptr, const int64_t *dims, float lo, float hi, int32_t nbins,
                    cube_stats_t *out, uint64_t *counts)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_sync(OP_FUSED, ptr, dims, lo, hi, nbins, out, counts);
    CUBE_GUARD_END
}

int cube_stats_hist_minmax(const float *ptr, const int64_t *dims, int32_t nbins,
                           cube_stats_t *out, uint64_t *counts)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_sync(OP_MINMAX, ptr, dims, 0.f, 0.f, nbins, out, counts);
    CUBE_GUARD_END
}

int cube_stats_async(const float *ptr, const int64_t *dims, cube_stats_t *dev_out,
                     void *stream)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_async_entry(OP_STATS, ptr, dims, 0.f, 0.f, 1, dev_out, nullptr, stream);
    CUBE_GUARD_END
}

int cube_hist_async(const float *ptr, const int64_t *dims, float lo, float hi, int32_t nbins,
                    uint64_t *dev_counts, void *stream)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_async_entry(OP_HIST, ptr, dims, lo, hi, nbins, nullptr, dev_counts, stream);
    CUBE_GUARD_END
}

int cube_stats_hist_async(const float *ptr, const int64_t *dims, float lo, float hi,
                          int32_t nbins, cube_stats_t *dev_out, uint64_t *dev_counts,
                          void *stream)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_async_entry(OP_FUSED, ptr, dims, lo, hi, nbins, dev_out, dev_counts, stream);
    CUBE_GUARD_END
}

int cube_stats_hist_minmax_async(const float *ptr, const int64_t *dims, int32_t nbins,
                                 cube_stats_t *dev_out, uint64_t *dev_counts, void *stream)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    return run_async_entry(OP_MINMAX, ptr, dims, 0.f, 0.f, nbins, dev_out, dev_counts, stream);
    CUBE_GUARD_END
}

int cube_set_accum_mode(int32_t mode)
{
    if (mode != CUBE_ACCUM_FP64MERGE && mode != CUBE_ACCUM_KAHAN32 && mode != CUBE_ACCUM_NAIVE32)
        return fail(CUBE_EINVAL, "unknown accumulation mode %d", mode);
    const int prev = g_accum;
    g_accum = mode;
    return prev;
}

int cube_set_hist_mode(int32_t mode)
{
    if (mode != CUBE_HIST_AUTO && mode != CUBE_HIST_PLAIN && mode != CUBE_HIST_HOT)
        return fail(CUBE_EINVAL, "unknown histogram form %d", mode);
    const int prev = g_hot < 0 ? CUBE_HIST_AUTO : (g_hot ? CUBE_HIST_HOT : CUBE_HIST_PLAIN);
    g_hot = mode == CUBE_HIST_AUTO ? -1 : (mode == CUBE_HIST_HOT ? 1 : 0);
    return prev;
}

int cube_describe_plan(const float *ptr, const int64_t *dims, int32_t kind, int32_t nbins,
                       char *out, size_t cap)
{
    CUBE_GUARD_BEGIN
    g_err.clear();
    if (kind != CUBE_Q_STATS && kind != CUBE_Q_HIST && kind != CUBE_Q_FUSED)
        return fail(CUBE_EINVAL, "plan kinds: CUBE_Q_STATS, CUBE_Q_HIST, CUBE_Q_FUSED");
    if (nbins < 1 || nbins > CUBE_MAX_BINS)
        return fail(CUBE_EINVAL, "nbins=%d outside [1, %d]", nbins, CUBE_MAX_BINS);
    if (!out || cap == 0) return fail(CUBE_EINVAL, "out is NULL or cap is 0");
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (rc) return rc;
    if ((rc = check_box_device(&b))) return rc;
    if (b.n == 0) return fail(CUBE_EINVAL, "an empty box launches nothing");
    Plan p;
    if ((rc = make_plan(b, kind != CUBE_Q_HIST, kind == CUBE_Q_STATS ? 0 : 1, nbins, &p)))
        return rc;
    static const char *forms[] = {"none", "lds", "global", "hot"};
    const int n = snprintf(out, cap,
                           "{\"threads\": %d, \"blocks\": %d, \"unroll\": %d, \"copies\": %d, "
                           "\"hist\": \"%s\", \"partition\": \"%s\", \"chunks\": %d, "
                           "\"units\": %lld}",
                           p.threads, p.blocks, p.unroll,
                           p.hist == HIST_NONE || p.hist == HIST_GLOBAL ? 0 : 1 << p.copies_log2,
                           forms[p.hist], p.chunks > 0 ? "dynamic" : "static", p.chunks,
                           (long long)p.g.n_units);
    if (n < 0 || (size_t)n >= cap) return fail(CUBE_EINVAL, "cap %zu too small for the plan", cap);
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_set_partition(int32_t chunk_log2)
{
    if (chunk_log2 != CUBE_PARTITION_AUTO && chunk_log2 != CUBE_PARTITION_STATIC &&
        (chunk_log2 < CUBE_CHUNK_LOG2_MIN || chunk_log2 > CUBE_CHUNK_LOG2_MAX))
        return fail(CUBE_EINVAL, "partition %d: 0 (automatic), 1 (static) or chunks of 2^k "
                    "voxels, k in [%d, %d]", chunk_log2, CUBE_CHUNK_LOG2_MIN, CUBE_CHUNK_LOG2_MAX);
    const int prev = g_chunk < 0 ? CUBE_PARTITION_AUTO
                                 : (g_chunk == 0 ? CUBE_PARTITION_STATIC : g_chunk);
    g_chunk = chunk_log2 == CUBE_PARTITION_AUTO ? -1
              : (chunk_log2 == CUBE_PARTITION_STATIC ? 0 : chunk_log2);
    return prev;
}

int cube_set_launch(int32_t threads, int32_t blocks, int32_t hist_copies, int32_t unroll)
{
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(CUBE_EINVAL, "threads must be 0, 256, 512 or 1024");
    if (blocks < 0 || blocks > MAX_BLOCKS) return fail(CUBE_EINVAL, "blocks outside [0, 4096]");
    if (hist_copies < 0 || hist_copies > 32 || (hist_copies & (hist_copies - 1)))
        return fail(CUBE_EINVAL, "hist_copies must be 0 or a power of two <= 32");
    if (unroll != 0 && unroll != 2 && unroll != 4)
        return fail(CUBE_EINVAL, "unroll must be 0, 2 or 4");
    g_threads = threads;
    g_blocks = blocks;
    g_copies = hist_copies;
    g_unroll = unroll;
    return CUBE_OK;
}

void cube_release_stream(void *stream)
{
    CUBE_GUARD_BEGIN
    release_ws((hipStream_t)stream);
    CUBE_GUARD_VOID_END
}

void cube_shutdown(void)
{
    CUBE_GUARD_BEGIN
    host_release();
    project_release();
    quant_release();
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_ws) free_ws(kv.second);
    g_ws.clear();
    CUBE_GUARD_VOID_END
}

}  // extern "C"
