// cube_host.hip -- out-of-core queries over cubes held in host memory.
//
// The paper's motivating cubes do not fit one device (a terabyte-scale
// survey cube, processed as many sub-cubes, Section 3), and its pipeline
// overlaps loading with processing (Section 2).  Here a cube in host memory
// is streamed through a ring of device buffers: a copy stream moves chunk i
// into buffer i mod NBUF while the compute stream runs the ordinary pass on
// chunk i-1.  Each chunk's pass leaves its own statistics record and adds its
// histogram counts to the running counts; a one-block kernel then merges the
// chunk records in chunk order (the pairwise FP64 update of Chan, Golub &
// LeVeque), so the result does not depend on timing.  A [min, max] histogram
// takes a second streaming pass that reads the merged range on the device.
//
// A chunk is a run of whole rows of one plane (or a piece of one row when a
// row alone exceeds the chunk), so a strided host box is gathered by one 2-D
// copy per chunk into a dense device buffer.
//
// Pinned host memory is copied by the DMA engine directly.  Pageable memory
// would go through the HIP runtime's own staging, one host thread at a time;
// here a few host threads gather each chunk (at most 64 MiB) into one of
// three pinned staging buffers while the DMA engine moves the previous one,
// and a staging buffer is reused only once the copy that read it is done.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <thread>
#include <vector>

#include "cube_device.h"

namespace cube {

namespace {

constexpr int NBUF = 3;
constexpr int64_t DEFAULT_CHUNK = (int64_t)1 << 28;  // voxels (1 GiB)
constexpr int64_t MIN_CHUNK = (int64_t)1 << 12;
constexpr int NSTAGE = 3;
constexpr int64_t STAGE_CHUNK = (int64_t)1 << 24;    // voxels (64 MiB) per staged chunk

// Merge per-chunk results in chunk order (one thread; the chunk count is
// small).  Writes the result and, when range_out is given, the [min, max]
// range exactly as a stats pass forms it.
__global__ void k_merge_chunks(const cube_stats_t *chunks, int n, unsigned long long n_total,
                               cube_stats_t *out, HistRange *range_out, int nbins)
{
    if (threadIdx.x != 0) return;
    double cnt = 0.0, mean = 0.0, m2 = 0.0;
    float mn = INFINITY, mx = -INFINITY;
    unsigned long long nv = 0;
    for (int i = 0; i < n; ++i) {
        const cube_stats_t c = chunks[i];
        if (c.n_valid == 0) continue;
        nv += c.n_valid;
        mn = fminf(mn, c.min);
        mx = fmaxf(mx, c.max);
        chan_merge<double>(cnt, mean, m2, (double)c.n_valid, c.mean, c.m2);
    }
    cube_stats_t o;
    o.n_total = n_total;
    o.n_valid = nv;
    o.n_nan = n_total - nv;
    o.flags = 0u;
    o.reserved = 0u;
    if (nv == 0) {
        o.min = o.max = qnan();
        o.mean = o.m2 = o.std = (double)qnan();
        o.flags |= CUBE_NO_VALID;
    } else {
        o.min = mn;
        o.max = mx;
        o.mean = mean;
        o.m2 = m2 < 0.0 ? 0.0 : m2;
        o.std = sqrt(o.m2 / (double)nv);
        extended_real_moments(o);
    }
    if (range_out) {
        const HistRange r = range_of_extrema(mn, mx, nv, nbins);
        if (r.ok == 0) o.flags |= CUBE_HIST_BAD_RANGE;
        *range_out = r;
    }
    *out = o;
}

__global__ void k_zero_counts(unsigned long long *counts, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) counts[i] = 0ull;
}

// One chunk: rows [y0, y0 + rows) of plane z, columns [c0, c0 + len).
struct Chunk {
    int64_t z, y0, rows, c0, len;
};

// Device-side state of the streaming path, one per device, grown on demand.
struct HostWorkspace {
    std::mutex mu;
    bool ready = false;
    hipStream_t copy = nullptr, compute = nullptr;
    hipEvent_t copied[NBUF] = {}, freed[NBUF] = {};
    float *buf[NBUF] = {};
    int64_t buf_voxels = 0;
    cube_stats_t *d_chunks = nullptr;
    size_t cap_chunks = 0;
    cube_stats_t *d_out = nullptr, *h_out = nullptr;
    unsigned long long *d_counts = nullptr, *h_counts = nullptr;
    HistRange *d_range = nullptr;
    // pinned staging of pageable sources
    float *stage[NSTAGE] = {};
    hipEvent_t stage_free[NSTAGE] = {};
};

HostWorkspace g_hws[64];
std::mutex g_hmu;

int hws_init(HostWorkspace &w)
{
    if (w.ready) return CUBE_OK;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&w.copy, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&w.compute, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "streaming streams");
    for (int i = 0; i < NBUF; ++i)
        if ((e = hipEventCreateWithFlags(&w.copied[i], hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&w.freed[i], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "streaming events");
    for (int i = 0; i < NSTAGE; ++i)
        if ((e = hipEventCreateWithFlags(&w.stage_free[i], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "staging events");
    if ((e = hipMalloc(&w.d_out, sizeof(cube_stats_t))) != hipSuccess ||
        (e = hipMalloc(&w.d_counts, ((size_t)CUBE_MAX_BINS + 3) * 8)) != hipSuccess ||
        (e = hipMalloc(&w.d_range, sizeof(HistRange))) != hipSuccess ||
        (e = hipHostMalloc(&w.h_out, sizeof(cube_stats_t))) != hipSuccess ||
        (e = hipHostMalloc(&w.h_counts, ((size_t)CUBE_MAX_BINS + 3) * 8)) != hipSuccess)
        return hip_fail(e, "streaming outputs");
    w.ready = true;
    return CUBE_OK;
}

int hws_reserve(HostWorkspace &w, int64_t chunk_voxels, size_t n_chunks)
{
    hipError_t e;
    if (chunk_voxels > w.buf_voxels) {
        for (int i = 0; i < NBUF; ++i) {
            hipFree(w.buf[i]);
            w.buf[i] = nullptr;
        }
        w.buf_voxels = 0;
        for (int i = 0; i < NBUF; ++i)
            if ((e = hipMalloc(&w.buf[i], (size_t)chunk_voxels * 4)) != hipSuccess)
                return hip_fail(e, "streaming buffers");
        w.buf_voxels = chunk_voxels;
    }
    if (n_chunks > w.cap_chunks) {
        hipFree(w.d_chunks);
        w.d_chunks = nullptr;
        w.cap_chunks = 0;
        const size_t cap = n_chunks < 64 ? 64 : n_chunks * 2;
        if ((e = hipMalloc(&w.d_chunks, cap * sizeof(cube_stats_t))) != hipSuccess)
            return hip_fail(e, "chunk records");
        w.cap_chunks = cap;
    }
    return CUBE_OK;
}

// Cut a collapsed box into chunks of at most `cv` voxels.
void plan_chunks(const Geom &g, int64_t cv, std::vector<Chunk> &out)
{
    out.clear();
    for (int64_t z = 0; z < g.nz; ++z) {
        if (g.row_len > cv) {
            for (int64_t y = 0; y < g.ny; ++y)
                for (int64_t c0 = 0; c0 < g.row_len; c0 += cv)
                    out.push_back(Chunk{z, y, 1, c0, std::min(cv, g.row_len - c0)});
        } else {
            const int64_t per = cv / g.row_len;
            for (int64_t y0 = 0; y0 < g.ny; y0 += per)
                out.push_back(Chunk{z, y0, std::min(per, g.ny - y0), 0, g.row_len});
        }
    }
}

// Gather rows [0, rows) of len floats at pitch sy from src into dense dst
// with up to `threads` host threads, each taking an equal share of the
// voxels.
void gather_rows(float *dst, const float *src, int64_t sy, int64_t rows, int64_t len,
                 int threads)
{
    const int64_t total = rows * len;
    auto part = [&](int t) {
        int64_t i = total * t / threads;
        const int64_t end = total * (t + 1) / threads;
        while (i < end) {
            const int64_t r = i / len, c = i - r * len;
            const int64_t n = std::min(len - c, end - i);
            memcpy(dst + i, src + r * sy + c, (size_t)n * 4);
            i += n;
        }
    };
    if (threads <= 1 || total < ((int64_t)1 << 18)) {
        threads = 1;
        part(0);
        return;
    }
    // A part whose thread cannot be started runs here instead (no exception
    // leaves the library).
    std::vector<std::thread> pool;
    int started = 1;
    try {
        for (int t = 1; t < threads; ++t, ++started) pool.emplace_back(part, t);
    } catch (...) {
    }
    for (int t = started; t < threads; ++t) part(t);
    part(0);
    for (std::thread &th : pool) th.join();
}

int gather_threads()
{
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(8u, hc / 2));
}

// One streaming pass over every chunk.  stats: per-chunk records into
// w.d_chunks; hist: counts added into w.d_counts over `range` or, when
// dev_range is set, the range on the device.  staged: the source is pageable
// and goes through the pinned staging buffers.
int stream_pass(HostWorkspace &w, const Geom &g, const std::vector<Chunk> &chunks, bool stats,
                bool hist, int nbins, const HistRange &range, const HistRange *dev_range,
                bool staged)
{
    hipError_t e;
    int rc;
    const int threads = staged ? gather_threads() : 1;
    for (size_t i = 0; i < chunks.size(); ++i) {
        const Chunk &c = chunks[i];
        const int k = (int)(i % NBUF);
        const float *src = g.ptr + c.z * g.sz + c.y0 * g.sy + c.c0;
        // The buffer is free once the pass that last read it has run.
        if ((e = hipStreamWaitEvent(w.copy, w.freed[k], 0)) != hipSuccess)
            return hip_fail(e, "wait for buffer");
        if (staged) {
            // The staging buffer is free once the copy that last read it is
            // done; then the host gathers the chunk into it.
            const int s = (int)(i % NSTAGE);
            if ((e = hipEventSynchronize(w.stage_free[s])) != hipSuccess)
                return hip_fail(e, "wait for staging");
            gather_rows(w.stage[s], src, g.sy, c.rows, c.len, threads);
            e = hipMemcpyAsync(w.buf[k], w.stage[s], (size_t)(c.len * c.rows) * 4,
                               hipMemcpyHostToDevice, w.copy);
            if (e == hipSuccess) e = hipEventRecord(w.stage_free[s], w.copy);
        } else if (c.rows == 1) {
            e = hipMemcpyAsync(w.buf[k], src, (size_t)c.len * 4, hipMemcpyHostToDevice, w.copy);
        } else {
            e = hipMemcpy2DAsync(w.buf[k], (size_t)c.len * 4, src, (size_t)g.sy * 4,
                                 (size_t)c.len * 4, (size_t)c.rows, hipMemcpyHostToDevice,
                                 w.copy);
        }
        if (e != hipSuccess) return hip_fail(e, "chunk copy");
        if ((e = hipEventRecord(w.copied[k], w.copy)) != hipSuccess)
            return hip_fail(e, "copy event");
        if ((e = hipStreamWaitEvent(w.compute, w.copied[k], 0)) != hipSuccess)
            return hip_fail(e, "wait for copy");
        Box b;
        b.ptr = w.buf[k];
        b.nx = c.len;
        b.ny = c.rows;
        b.nz = 1;
        b.sy = c.len;
        b.sz = c.len * c.rows;
        b.n = (uint64_t)(c.len * c.rows);
        if ((rc = run_pass(b, stats, hist, nbins, range, dev_range,
                           stats ? w.d_chunks + i : nullptr, w.d_counts, true, w.compute)))
            return rc;
        if ((e = hipEventRecord(w.freed[k], w.compute)) != hipSuccess)
            return hip_fail(e, "compute event");
    }
    return CUBE_OK;
}

int host_query(const cube_query_t *q, int64_t chunk_voxels)
{
    if (!q) return fail(CUBE_EINVAL, "query is NULL");
    const int kind = q->kind;
    if (kind != CUBE_Q_STATS && kind != CUBE_Q_HIST && kind != CUBE_Q_FUSED &&
        kind != CUBE_Q_MINMAX)
        return fail(CUBE_EINVAL, "unknown query kind %d", kind);
    const bool want_stats = kind != CUBE_Q_HIST, want_hist = kind != CUBE_Q_STATS;
    if (want_stats && !q->out) return fail(CUBE_EINVAL, "stats output is NULL");
    if (want_hist && !q->counts) return fail(CUBE_EINVAL, "counts output is NULL");
    if (chunk_voxels == 0) chunk_voxels = DEFAULT_CHUNK;
    if (chunk_voxels < MIN_CHUNK || chunk_voxels > ((int64_t)1 << 31))
        return fail(CUBE_EINVAL, "chunk_voxels=%lld outside [2^12, 2^31]",
                    (long long)chunk_voxels);
    chunk_voxels &= ~(int64_t)3;
    Box box;
    int rc = check_box(q->ptr, q->dims, &box);
    if (rc) return rc;
    HistRange range = {0.f, 0.f, 0.f, 1};
    int nbins = 1;
    if (want_hist) {
        nbins = q->nbins;
        if (kind == CUBE_Q_MINMAX) {
            if (nbins < 1 || nbins > CUBE_MAX_BINS)
                return fail(CUBE_EINVAL, "nbins=%d outside [1, %d]", nbins, CUBE_MAX_BINS);
        } else if ((rc = check_range(q->lo, q->hi, nbins, &range))) {
            return rc;
        }
    }
    // The input must be host memory: device memory takes the resident path.
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    const bool known = hipPointerGetAttributes(&attr, q->ptr) == hipSuccess;
    if (known && attr.type == hipMemoryTypeDevice)
        return fail(CUBE_EINVAL, "the box is in device memory: use the resident entry points");
    (void)hipGetLastError();  // a pageable pointer leaves an error code behind
    // Pinned (registered) host memory is copied directly; anything else is
    // staged.
    const bool staged = !(known && attr.type == hipMemoryTypeHost);
    if (staged) chunk_voxels = std::min(chunk_voxels, STAGE_CHUNK);
    int dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "device");
    if (dev < 0 || dev >= 64) return fail(CUBE_EINVAL, "device index out of range");
    HostWorkspace &w = g_hws[dev];
    std::lock_guard<std::mutex> lk(w.mu);
    {
        std::lock_guard<std::mutex> gl(g_hmu);
        if ((rc = hws_init(w))) return rc;
    }
    Geom g;
    collapse(box, &g);
    std::vector<Chunk> chunks;
    if (box.n) plan_chunks(g, chunk_voxels, chunks);
    if ((rc = hws_reserve(w, std::min<int64_t>(chunk_voxels, (int64_t)box.n + 4),
                          chunks.size())))
        return rc;
    if (staged && box.n && !w.stage[0])
        for (int i = 0; i < NSTAGE; ++i)
            if ((e = hipHostMalloc(&w.stage[i], (size_t)STAGE_CHUNK * 4)) != hipSuccess)
                return hip_fail(e, "staging buffers");
    // Every buffer starts free.
    for (int k = 0; k < NBUF; ++k)
        if ((e = hipEventRecord(w.freed[k], w.compute)) != hipSuccess)
            return hip_fail(e, "initial events");
    for (int i = 0; i < NSTAGE; ++i)
        if ((e = hipEventRecord(w.stage_free[i], w.copy)) != hipSuccess)
            return hip_fail(e, "initial events");
    if (box.n == 0) {
        if ((rc = write_empty(w.d_out, w.d_counts, nbins, w.compute))) return rc;
    } else {
        if (want_hist) {
            hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1024), 0, w.compute, w.d_counts,
                               nbins + 3);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "zero counts");
        }
        const bool fused_pass = kind != CUBE_Q_MINMAX;
        if ((rc = stream_pass(w, g, chunks, want_stats, want_hist && fused_pass, nbins, range,
                              nullptr, staged)))
            return rc;
        if (want_stats) {
            hipLaunchKernelGGL(k_merge_chunks, dim3(1), dim3(64), 0, w.compute, w.d_chunks,
                               (int)chunks.size(), (unsigned long long)box.n, w.d_out,
                               kind == CUBE_Q_MINMAX ? w.d_range : nullptr, nbins);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "chunk merge");
        }
        if (kind == CUBE_Q_MINMAX &&
            (rc = stream_pass(w, g, chunks, false, true, nbins, range, w.d_range, staged)))
            return rc;
    }
    if (want_stats &&
        (e = hipMemcpyAsync(w.h_out, w.d_out, sizeof(cube_stats_t), hipMemcpyDeviceToHost,
                            w.compute)) != hipSuccess)
        return hip_fail(e, "result copy");
    if (want_hist &&
        (e = hipMemcpyAsync(w.h_counts, w.d_counts, ((size_t)nbins + 3) * 8,
                            hipMemcpyDeviceToHost, w.compute)) != hipSuccess)
        return hip_fail(e, "counts copy");
    if ((e = hipStreamSynchronize(w.compute)) != hipSuccess) return hip_fail(e, "synchronize");
    if ((e = hipStreamSynchronize(w.copy)) != hipSuccess) return hip_fail(e, "synchronize");
    if (want_stats) *q->out = *w.h_out;
    if (want_hist) memcpy(q->counts, w.h_counts, ((size_t)nbins + 3) * 8);
    if (kind == CUBE_Q_MINMAX && (w.h_out->flags & CUBE_HIST_BAD_RANGE))
        return fail(CUBE_EINVAL, "the data range [min, max] is not a valid histogram range");
    return CUBE_OK;
}

}  // namespace

void host_release()
{
    for (HostWorkspace &w : g_hws) {
        std::lock_guard<std::mutex> lk(w.mu);
        if (!w.ready) continue;
        hipStreamSynchronize(w.compute);
        hipStreamSynchronize(w.copy);
        for (int i = 0; i < NBUF; ++i) {
            hipFree(w.buf[i]);
            w.buf[i] = nullptr;
            hipEventDestroy(w.copied[i]);
            hipEventDestroy(w.freed[i]);
        }
        for (int i = 0; i < NSTAGE; ++i) {
            hipHostFree(w.stage[i]);
            w.stage[i] = nullptr;
            hipEventDestroy(w.stage_free[i]);
        }
        w.buf_voxels = 0;
        hipFree(w.d_chunks);
        w.d_chunks = nullptr;
        w.cap_chunks = 0;
        hipFree(w.d_out);
        hipFree(w.d_counts);
        hipFree(w.d_range);
        hipHostFree(w.h_out);
        hipHostFree(w.h_counts);
        release_ws(w.compute);  // the passes' workspace on the compute stream
        hipStreamDestroy(w.copy);
        hipStreamDestroy(w.compute);
        w.copy = w.compute = nullptr;
        w.d_out = w.h_out = nullptr;
        w.d_counts = w.h_counts = nullptr;
        w.d_range = nullptr;
        w.ready = false;
    }
}

}  // namespace cube

extern "C" {

int cube_host_query(const cube_query_t *q, int64_t chunk_voxels)
{
    CUBE_GUARD_BEGIN
    return cube::host_query(q, chunk_voxels);
    CUBE_GUARD_END
}

}  // extern "C"
