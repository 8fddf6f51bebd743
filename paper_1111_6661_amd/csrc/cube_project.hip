// cube_project.hip -- projections of a cube along its channel axis.
//
// The case study renders spectral cubes for inspection (Section 2); the maps a
// viewer shows beside the volume reduce the channel axis of every spatial
// pixel: the maximum-intensity projection, the sum of the channels (the
// moment-0 map up to the channel width) and the number of valid channels.
// One streaming read of the cube makes all three.
//
// When the rows are contiguous and 16-byte aligned, lanes own quads of pixels
// numbered over the whole image, Q quads per lane 1 KB apart, so that per
// channel a wavefront reads Q KB of contiguous memory (k_project_quads).
// Otherwise each lane owns V adjacent pixels of one row (V = 4 when rows,
// planes and the base are 16-byte aligned, else 1), four channels in flight
// (k_project).  Each lane walks the channels of its pixels.  The
// sums are taken in FP64: on CDNA4 an FP64 add issues at the rate of an FP32
// add, so this costs no more than compensated FP32 and is exact to about
// n * 2^-53.  When the image has too few pixels to fill the device the
// channels are split into slices, each slice writes per-pixel partials, and a
// second kernel merges them in slice order, so the result never depends on
// timing.
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include "cube_device.h"

namespace cube {

namespace {

struct ProjArgs {
    const float *ptr;
    int64_t nx, ny, nz, sy, sz;
    int64_t units;           // lanes' work items: pixels (V = 1) or quads (V = 4)
    int64_t u0;              // k_project: first unit; k_project_quads: units it covers
    int64_t zps;             // channels per slice
    int32_t slices;
    float *mip;              // outputs, dense nx * ny (any may be null)
    double *mom0;
    uint32_t *nvalid;
    float *p_max;            // slice partials [slices][npix] (slices > 1)
    double *p_sum;
    uint32_t *p_cnt;
};

constexpr int PROJ_THREADS = 256;
constexpr int PROJ_ZU = 4;

template <int V>
__global__ void __launch_bounds__(PROJ_THREADS) k_project(ProjArgs a)
{
    const int64_t u = a.u0 + (int64_t)blockIdx.x * PROJ_THREADS + threadIdx.x;
    if (u >= a.units) return;
    const int64_t row_units = a.nx / V;
    const int64_t y = u / row_units;
    const int64_t x = (u - y * row_units) * V;
    const int64_t z0 = (int64_t)blockIdx.y * a.zps;
    const int64_t z1 = min(a.nz, z0 + a.zps);
    const float *q = a.ptr + y * a.sy + x + z0 * a.sz;
    float m[V];
    double s[V];
    uint32_t n[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        m[k] = -INFINITY;
        s[k] = 0.0;
        n[k] = 0u;
    }
    auto take = [&](const float (&v)[V]) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool ok = v[k] == v[k];
            m[k] = ok ? fmaxf(m[k], v[k]) : m[k];
            s[k] += (double)(ok ? v[k] : 0.f);
            n[k] += ok ? 1u : 0u;
        }
    };
    auto load = [&](const float *p, float (&v)[V]) {
        if constexpr (V == 4) {
            const f4 t = __builtin_nontemporal_load((const f4 *)p);
            v[0] = t.x;
            v[1] = t.y;
            v[2] = t.z;
            v[3] = t.w;
        } else {
            v[0] = __builtin_nontemporal_load(p);
        }
    };
    int64_t z = z0;
    for (; z + PROJ_ZU <= z1; z += PROJ_ZU) {
        float v[PROJ_ZU][V];
#pragma unroll
        for (int j = 0; j < PROJ_ZU; ++j) load(q + j * a.sz, v[j]);
#pragma unroll
        for (int j = 0; j < PROJ_ZU; ++j) take(v[j]);
        q += PROJ_ZU * a.sz;
    }
    for (; z < z1; ++z) {
        float v[V];
        load(q, v);
        take(v);
        q += a.sz;
    }
    const int64_t p = y * a.nx + x;
    if (a.slices == 1) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (a.mip) a.mip[p + k] = n[k] ? m[k] : qnan();
            if (a.mom0) a.mom0[p + k] = n[k] ? s[k] : (double)qnan();
            if (a.nvalid) a.nvalid[p + k] = n[k];
        }
    } else {
        const int64_t o = (int64_t)blockIdx.y * a.nx * a.ny + p;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            a.p_max[o + k] = m[k];
            a.p_sum[o + k] = s[k];
            a.p_cnt[o + k] = n[k];
        }
    }
}

// The fast path for images whose rows are contiguous and 16-byte aligned:
// pixel quads are numbered over the whole image, and wavefront w owns quads
// [64 Q w, 64 Q (w + 1)), lane l the quads 64 k + l.  Per channel a wavefront
// then reads Q runs of 1 KB that together cover 1 KB * Q of contiguous
// memory, which keeps HBM pages open far better than 1 KB per wavefront.
template <int Q>
__global__ void __launch_bounds__(PROJ_THREADS) k_project_quads(ProjArgs a)
{
    // Launched for whole wavefronts only; the remaining quads go to k_project.
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * PROJ_THREADS + threadIdx.x) >> 6;
    const int64_t qb = wave * 64 * Q;
    if (qb + 64 * Q > a.u0) return;
    const int64_t z0 = (int64_t)blockIdx.y * a.zps;
    const int64_t z1 = min(a.nz, z0 + a.zps);
    const int64_t sz4 = a.sz >> 2;
    const f4 *q = (const f4 *)a.ptr + qb + lane + z0 * sz4;
    float m[Q][4];
    double s[Q][4];
    uint32_t n[Q][4];
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            m[k][j] = -INFINITY;
            s[k][j] = 0.0;
            n[k][j] = 0u;
        }
    for (int64_t z = z0; z < z1; ++z) {
        f4 v[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) v[k] = __builtin_nontemporal_load(q + 64 * k);
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float x = v[k][j];
                const bool ok = x == x;
                m[k][j] = ok ? fmaxf(m[k][j], x) : m[k][j];
                s[k][j] += (double)(ok ? x : 0.f);
                n[k][j] += ok ? 1u : 0u;
            }
        q += sz4;
    }
    const int64_t o = a.slices == 1 ? 0 : (int64_t)blockIdx.y * a.nx * a.ny;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int64_t p = (qb + 64 * k + lane) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (a.slices == 1) {
                if (a.mip) a.mip[p + j] = n[k][j] ? m[k][j] : qnan();
                if (a.mom0) a.mom0[p + j] = n[k][j] ? s[k][j] : (double)qnan();
                if (a.nvalid) a.nvalid[p + j] = n[k][j];
            } else {
                a.p_max[o + p + j] = m[k][j];
                a.p_sum[o + p + j] = s[k][j];
                a.p_cnt[o + p + j] = n[k][j];
            }
        }
    }
}

// Merge the slice partials of every pixel in slice order.
__global__ void __launch_bounds__(PROJ_THREADS) k_project_merge(ProjArgs a)
{
    const int64_t npix = a.nx * a.ny;
    const int64_t p = (int64_t)blockIdx.x * PROJ_THREADS + threadIdx.x;
    if (p >= npix) return;
    float m = -INFINITY;
    double s = 0.0;
    uint32_t n = 0u;
    for (int k = 0; k < a.slices; ++k) {
        const int64_t o = (int64_t)k * npix + p;
        m = fmaxf(m, a.p_max[o]);
        s += a.p_sum[o];
        n += a.p_cnt[o];
    }
    if (a.mip) a.mip[p] = n ? m : qnan();
    if (a.mom0) a.mom0[p] = n ? s : (double)qnan();
    if (a.nvalid) a.nvalid[p] = n;
}

__global__ void k_project_empty(ProjArgs a)
{
    const int64_t npix = a.nx * a.ny;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (a.mip) a.mip[p] = qnan();
        if (a.mom0) a.mom0[p] = (double)qnan();
        if (a.nvalid) a.nvalid[p] = 0u;
    }
}

// Slice partials, one buffer per (device, stream), grown on demand.
struct ProjScratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_pmu;
std::map<std::pair<int, hipStream_t>, ProjScratch> g_pscratch;

int scratch_for(hipStream_t s, size_t bytes, void **out)
{
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_pmu);
    ProjScratch &ps = g_pscratch[std::make_pair(dev, s)];
    if (ps.bytes < bytes) {
        hipError_t e;
        // Earlier work on this stream may still read the old buffer.
        if (ps.ptr && (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "projection scratch");
        hipFree(ps.ptr);
        ps.ptr = nullptr;
        ps.bytes = 0;
        if ((e = hipMalloc(&ps.ptr, bytes)) != hipSuccess)
            return hip_fail(e, "projection scratch");
        ps.bytes = bytes;
    }
    *out = ps.ptr;
    return CUBE_OK;
}

// An output map must be device memory holding `bytes`, aligned to `align`.
int check_output(const void *p, size_t bytes, uintptr_t align, const char *what)
{
    if (!p) return CUBE_OK;
    if ((uintptr_t)p % align)
        return fail(CUBE_EINVAL, "%s is not %d-byte aligned", what, (int)align);
    Box b;
    b.ptr = (const float *)p;
    b.nx = (int64_t)(bytes / 4);
    b.ny = b.nz = 1;
    b.sy = b.nx;
    b.sz = b.nx;
    b.n = (uint64_t)b.nx;
    const int rc = check_box_device(&b);
    if (rc) return fail(rc, "%s: %s", what, cube_last_error());
    return CUBE_OK;
}

}  // namespace

void project_release()
{
    std::lock_guard<std::mutex> lk(g_pmu);
    int cur = 0;
    hipGetDevice(&cur);
    for (auto &kv : g_pscratch) {
        // The stream may be gone: wait for the whole device instead.
        hipSetDevice(kv.first.first);
        hipDeviceSynchronize();
        hipFree(kv.second.ptr);
    }
    hipSetDevice(cur);
    g_pscratch.clear();
}

}  // namespace cube

using namespace cube;

extern "C" {

int cube_project(const float *ptr, const int64_t *dims, float *mip, double *mom0,
                 uint32_t *nvalid, void *stream)
{
    CUBE_GUARD_BEGIN
    if (!mip && !mom0 && !nvalid) return fail(CUBE_EINVAL, "every output is NULL");
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (rc) return rc;
    if (b.nz >= ((int64_t)1 << 32)) return fail(CUBE_EINVAL, "more than 2^32 - 1 channels");
    const int64_t npix = b.nx * b.ny;
    if (npix == 0) return CUBE_OK;
    if ((rc = check_output(mip, (size_t)npix * 4, 4, "mip")) ||
        (rc = check_output(mom0, (size_t)npix * 8, 8, "mom0")) ||
        (rc = check_output(nvalid, (size_t)npix * 4, 4, "nvalid")))
        return rc;
    if ((rc = check_box_device(&b))) return rc;
    hipStream_t s = (hipStream_t)stream;
    ProjArgs a;
    memset(&a, 0, sizeof a);
    a.ptr = b.ptr;
    a.nx = b.nx;
    a.ny = b.ny;
    a.nz = b.nz;
    a.sy = b.ny > 1 ? b.sy : b.nx;
    a.sz = b.nz > 1 ? b.sz : 0;
    a.mip = mip;
    a.mom0 = mom0;
    a.nvalid = nvalid;
    hipError_t e;
    if (b.nz == 0) {
        hipLaunchKernelGGL(k_project_empty, dim3(1024), dim3(256), 0, s, a);
        e = hipGetLastError();
        return e == hipSuccess ? CUBE_OK : hip_fail(e, "projection launch");
    }
    // Quads when every row start is 16-byte aligned; whole-image quads when,
    // in addition, the rows follow each other in memory.
    const bool quad = (b.nx % 4 == 0) && ((uintptr_t)b.ptr % 16 == 0) &&
                      (b.ny == 1 || a.sy % 4 == 0) && (b.nz == 1 || a.sz % 4 == 0);
    const bool rows = quad && (b.ny == 1 || a.sy == b.nx);
    const int V = quad ? 4 : 1;
    a.units = npix / V;
    // Quads per lane on the fast path: the most that still leaves about four
    // wavefronts per CU (each holds Q * 16 pixels of state in registers).
    const int64_t cus = cu_count();
    int Q = 1;
    if (rows) {
        Q = 4;
        if ((a.units + 64 * 16 - 1) / (64 * 16) >= 4 * cus) Q = 16;
        else if ((a.units + 64 * 8 - 1) / (64 * 8) >= 4 * cus) Q = 8;
    }
    // Slices of the channel axis until enough wavefronts are busy (16 per CU
    // on the general path, 4 on the fast path), each slice keeping at least
    // 64 channels.
    const int64_t waves = (a.units + 64 * Q - 1) / (64 * Q);
    const int64_t want = cus * (rows ? 4 : 16);
    int64_t slices = waves >= want ? 1 : (want + waves - 1) / waves;
    slices = std::min<int64_t>(slices, std::max<int64_t>(1, b.nz / 64));
    slices = std::min<int64_t>(slices, 64);
    a.zps = (b.nz + slices - 1) / slices;
    a.slices = (int32_t)((b.nz + a.zps - 1) / a.zps);
    if (a.slices > 1) {
        void *scr = nullptr;
        const size_t per = (size_t)npix * (size_t)a.slices;
        if ((rc = scratch_for(s, per * 16, &scr))) return rc;
        a.p_sum = (double *)scr;
        a.p_max = (float *)((char *)scr + per * 8);
        a.p_cnt = (uint32_t *)((char *)scr + per * 12);
    }
    // Whole wavefronts of the fast path first, then every remaining unit on
    // the general kernel (all of them when the fast path does not apply).
    int64_t done = 0;
    if (rows) {
        const int64_t full = a.units / (64 * Q);
        done = full * 64 * Q;
        if (full) {
            a.u0 = done;
            const dim3 grid((unsigned)((full * 64 + PROJ_THREADS - 1) / PROJ_THREADS),
                            (unsigned)a.slices);
            if (Q == 16)
                hipLaunchKernelGGL(k_project_quads<16>, grid, dim3(PROJ_THREADS), 0, s, a);
            else if (Q == 8)
                hipLaunchKernelGGL(k_project_quads<8>, grid, dim3(PROJ_THREADS), 0, s, a);
            else
                hipLaunchKernelGGL(k_project_quads<4>, grid, dim3(PROJ_THREADS), 0, s, a);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "projection launch");
        }
    }
    if (done < a.units) {
        a.u0 = done;
        const dim3 grid((unsigned)((a.units - done + PROJ_THREADS - 1) / PROJ_THREADS),
                        (unsigned)a.slices);
        if (quad)
            hipLaunchKernelGGL(k_project<4>, grid, dim3(PROJ_THREADS), 0, s, a);
        else
            hipLaunchKernelGGL(k_project<1>, grid, dim3(PROJ_THREADS), 0, s, a);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "projection launch");
    if (a.slices > 1) {
        hipLaunchKernelGGL(k_project_merge, dim3((unsigned)((npix + PROJ_THREADS - 1) / PROJ_THREADS)),
                           dim3(PROJ_THREADS), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "projection merge");
    }
    return CUBE_OK;
    CUBE_GUARD_END
}

}  // extern "C"
