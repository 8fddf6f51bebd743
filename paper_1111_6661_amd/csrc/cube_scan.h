// cube_scan.h -- pieces shared by the selection kernels (k-th smallest,
// median and quantiles): the order-preserving 32-bit key of a float and a
// visit of every voxel of a box in the single-box passes' layout.
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

// Visit every voxel of the box once, in tiles of float4 loads; `step` is
// called with arrays of 1, 4 or 4 * SEL_U voxels (blank lanes padded with
// NaN), uniformly across each wavefront.
template <class Step>
__device__ __forceinline__ void scan_box(const Geom &g, Step &step)
{
    const int tid = threadIdx.x, B = blockDim.x;
    const unsigned long long G = gridDim.x;
    const long long u0 = (long long)(((unsigned long long)g.n_units * blockIdx.x) / G);
    const long long u1 = (long long)(((unsigned long long)g.n_units * (blockIdx.x + 1)) / G);
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

// The geometry of a selection pass over a validated box: rows cut into
// segments so that `blocks` blocks get at least one work unit each.
inline void scan_geom(const Box &b, int blocks, Geom *g)
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

}  // namespace cube
