// cube_scan.h -- pieces shared by the selection kernels (k-th smallest,
// median and quantiles): the order-preserving 32-bit key of a float, a visit
// of every voxel of a box in the single-box passes' layout, and the static or
// dynamic partition of that visit among the blocks.
#pragma once

#include "cube_device.h"

namespace cube {

constexpr int SEL_U = 4;

__device__ __forceinline__ unsigned int order_key(float x)
{
    const unsigned int u = __float_as_uint(x);
    return u ^ ((unsigned int)((int)u >> 31) | 0x80000000u);
}

__device__ __forceinline__ float key_value(unsigned int k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Visit the work units [u0, u1) of a box once, in tiles of float4 loads;
// `step` is called with arrays of 1, 4 or 4 * SEL_U voxels (blank lanes
// padded with NaN), uniformly across each wavefront.
template <class Step>
__device__ __forceinline__ void scan_units_of(const Geom &g, long long u0, long long u1,
                                              Step &step)
{
    const int tid = threadIdx.x, B = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6;
    if (u0 >= u1) return;
    long long row = u0 / g.segs;
    long long s = u0 - row * g.segs;
    long long y = row % g.ny;
    long long z = row / g.ny;
    for (long long u = u0; u < u1; ++u) {
        const float *q = g.ptr + y * g.sy + z * g.sz + s * g.seg_len;
        const long long c0 = s * g.seg_len;
        const long long len = min(g.seg_len, g.row_len - c0);
        const long long mis = (long long)((16 - ((uintptr_t)q & 15)) & 15) >> 2;
        const long long h = min(len, mis);
        const long long n4 = (len - h) >> 2;
        const long long t = len - h - 4 * n4;
        if (wid == 0 && h + t > 0) {
            long long idx = lane < h ? lane : h + 4 * n4 + (lane - h);
            const bool have = lane < h + t;
            idx = have ? idx : 0;
            const float v = q[idx];
            float xv[1] = {have ? v : qnan()};
            step(xv);
        }
        const f4 *q4 = (const f4 *)(q + h);
        const long long T = (long long)B * SEL_U;
        long long i0 = 0;
        for (; i0 + T <= n4; i0 += T) {
            f4 v[SEL_U];
            load_tile<SEL_U>(v, q4, i0, B, tid);
            float xv[4 * SEL_U];
#pragma unroll
            for (int k = 0; k < SEL_U; ++k) {
                xv[4 * k + 0] = v[k].x;
                xv[4 * k + 1] = v[k].y;
                xv[4 * k + 2] = v[k].z;
                xv[4 * k + 3] = v[k].w;
            }
            step(xv);
        }
        for (; i0 < n4; i0 += B) {
            const long long i = i0 + tid;
            const bool have = i < n4;
            const f4 v = __builtin_nontemporal_load(q4 + (have ? i : n4 - 1));
            float xv[4] = {have ? v.x : qnan(), have ? v.y : qnan(), have ? v.z : qnan(),
                           have ? v.w : qnan()};
            step(xv);
        }
        if (++s == g.segs) {
            s = 0;
            if (++y == g.ny) {
                y = 0;
                ++z;
            }
        }
    }
}

// How a pass divides the box among its blocks: nc == 0, one contiguous range
// of work units per block (static); else nc chunks of consecutive units that
// the blocks claim from the counter *ctr (0 at launch; the pass returns it to
// 0), the next one as a chunk starts unless fewer than two grids' worth
// remain -- the single-box pass's dynamic partition.  The steps only count,
// so the partition does not change any result.
struct Claim {
    unsigned int *ctr;
    int nc;
};

// Visit every voxel of the box once (called by every thread of the block).
template <class Step>
__device__ __forceinline__ void scan_box(const Geom &g, Step &step, const Claim &cl)
{
    if (cl.nc <= 0) {
        const unsigned long long G = gridDim.x;
        const long long u0 = (long long)(((unsigned long long)g.n_units * blockIdx.x) / G);
        const long long u1 = (long long)(((unsigned long long)g.n_units * (blockIdx.x + 1)) / G);
        scan_units_of(g, u0, u1, step);
        return;
    }
    __shared__ int s_chunk;
    const int tid = threadIdx.x;
    if (tid == 0) s_chunk = (int)atomicAdd(cl.ctr, 1u);
    __syncthreads();
    while (true) {
        const int c = s_chunk;
        if (c >= cl.nc) break;
        const bool early = (long long)c + 2ll * gridDim.x < (long long)cl.nc;
        unsigned int next = 0u;
        if (tid == 0 && early) next = atomicAdd(cl.ctr, 1u);
        const long long u0 = (long long)(((unsigned long long)g.n_units * c) / cl.nc);
        const long long u1 = (long long)(((unsigned long long)g.n_units * (c + 1)) / cl.nc);
        scan_units_of(g, u0, u1, step);
        __syncthreads();  // every thread has read s_chunk
        if (tid == 0) s_chunk = (int)(early ? next : atomicAdd(cl.ctr, 1u));
        __syncthreads();
    }
}

// The geometry of a selection pass over a validated box: rows cut into
// segments so that there are at least `blocks` work units (one per block,
// or one per chunk of a dynamic partition).
inline void scan_geom(const Box &b, long long blocks, Geom *g)
{
    collapse(b, g);
    const long long rows = g->ny * g->nz;
    const long long segs = rows < blocks ? (blocks + rows - 1) / rows : 1;
    long long seg_len = ((g->row_len + segs - 1) / segs + 3) & ~3LL;
    if (seg_len < 4) seg_len = 4;
    g->seg_len = seg_len;
    g->segs = (g->row_len + seg_len - 1) / seg_len;
    g->n_units = rows * g->segs;
}

// The chunk size (log2 voxels; 0: static) of a selection pass over box b:
// the calling thread's cube_set_partition setting, where automatic means
// chunks of 2^18 voxels from 2^27 voxels on (as for the histogram passes).
inline int scan_chunk_log2(const Box &b)
{
    const int cl = chunk_override();
    if (cl >= 0) return cl;
    return b.n >= ((uint64_t)1 << 27) ? 18 : 0;
}

// The partition of a selection pass over box b with kernel k (`threads` per
// block, `lds` dynamic LDS bytes).  Static: two blocks per CU, *chunks = 0.
// Dynamic: one resident wave of blocks over chunks_of(n, scan_chunk_log2).
inline int scan_plan(const Box &b, const void *k, int threads, size_t lds, int *blocks,
                     int *chunks)
{
    const int cl = scan_chunk_log2(b);
    *chunks = 0;
    *blocks = cu_count() * 2;
    if (cl == 0) return CUBE_OK;
    hipError_t e;
    if (lds > 64 * 1024 &&
        (e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
            hipSuccess)
        return hip_fail(e, "selection LDS");
    int fit = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, k, threads, lds)) != hipSuccess)
        return hip_fail(e, "selection occupancy");
    const long long nc = chunks_of(b.n, cl);
    long long g = (long long)cu_count() * (fit < 1 ? 1 : fit);
    if (g > nc) g = nc;
    *blocks = (int)g;
    *chunks = (int)nc;
    return CUBE_OK;
}

}  // namespace cube
