// cube_probe.hip -- the read ceiling of the fused pass's access pattern.
//
// The fused statistics-and-histogram pass is bound by HBM reads.  To know
// how close it comes to what its own access pattern can reach, k_probe reads
// the same box in the same launch shape (grid, block size, dynamic LDS, and
// so the same resident blocks when registers allow) and in the same order: the
// same work units per block, the same software-pipelined tiles of U float4
// loads per lane with non-temporal hints, the same head and tail voxels.  Per
// voxel it does one bitwise OR, so its time is the read time of that pattern.
// The OR of every voxel's bit pattern is its result, which keeps every load
// alive and can be checked exactly.
#include <string.h>

#include "cube_device.h"

namespace cube {

namespace {

template <int U>
__device__ __forceinline__ unsigned int or_tile(const f4 (&v)[U])
{
    unsigned int r = 0u;
#pragma unroll
    for (int k = 0; k < U; ++k)
        r |= __float_as_uint(v[k].x) | __float_as_uint(v[k].y) | __float_as_uint(v[k].z) |
             __float_as_uint(v[k].w);
    return r;
}

// The OR of the bit patterns of work units [u0, u1), read in the fused
// pass's order and tiles.
template <int U>
__device__ __forceinline__ unsigned int or_units(const Geom &g, long long u0, long long u1)
{
    const int tid = threadIdx.x, B = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6;
    unsigned int acc = 0u;
    if (u0 >= u1) return acc;
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
        if (wid == 0 && lane < h + t) {
            // Head voxels are lanes [0, h), tail voxels lanes [h, h + t).
            const long long idx = lane < h ? lane : h + 4 * n4 + (lane - h);
            acc |= __float_as_uint(q[idx]);
        }
        const f4 *q4 = (const f4 *)(q + h);
        const long long T = (long long)B * U;
        const long long ntiles = n4 / T;
        if (ntiles > 0) {
            f4 va[U], vb[U];
            load_tile<U>(va, q4, 0, B, tid);
            long long k = 0;
            while (true) {
                if (k + 1 < ntiles) load_tile<U>(vb, q4, (k + 1) * T, B, tid);
                acc |= or_tile<U>(va);
                if (++k == ntiles) break;
                if (k + 1 < ntiles) load_tile<U>(va, q4, (k + 1) * T, B, tid);
                acc |= or_tile<U>(vb);
                if (++k == ntiles) break;
            }
        }
        for (long long i = ntiles * T + tid; i < n4; i += B) {
            const f4 v = __builtin_nontemporal_load(q4 + i);
            acc |= __float_as_uint(v.x) | __float_as_uint(v.y) | __float_as_uint(v.z) |
                   __float_as_uint(v.w);
        }
        if (++s == g.segs) {
            s = 0;
            if (++y == g.ny) {
                y = 0;
                ++z;
            }
        }
    }
    return acc;
}

// One atomic per block, as the fused pass takes one ticket per block.
__device__ __forceinline__ void or_out(unsigned int acc, unsigned int *out)
{
    __shared__ unsigned int s_or[MAX_WAVES];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int o = 32; o > 0; o >>= 1) acc |= (unsigned int)__shfl_xor((int)acc, o, 64);
    if (lane == 0) s_or[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int r = 0u;
        for (int w = 0; w < nw; ++w) r |= s_or[w];
        atomicOr(out, r);
    }
}

template <int U>
__global__ void __launch_bounds__(1024) k_probe(Geom g, unsigned int *out)
{
    const unsigned long long G = gridDim.x;
    const long long u0 = (long long)(((unsigned long long)g.n_units * blockIdx.x) / G);
    const long long u1 = (long long)(((unsigned long long)g.n_units * (blockIdx.x + 1)) / G);
    or_out(or_units<U>(g, u0, u1), out);
}

// The same read with the fused pass's dynamic partition: chunks claimed from
// the counter `ctr` (0 at launch) with the same early claim and the same two
// barriers per chunk; the last block returns the counter to 0.
template <int U>
__global__ void __launch_bounds__(1024) k_probe_dyn(Geom g, unsigned int *out, unsigned int *ctr,
                                                    int nc)
{
    __shared__ int s_chunk;
    __shared__ unsigned int s_last;
    const int tid = threadIdx.x;
    unsigned int acc = 0u;
    if (tid == 0) s_chunk = (int)atomicAdd(&ctr[0], 1u);
    __syncthreads();
    while (true) {
        const int c = s_chunk;
        if (c >= nc) break;
        const bool early = (long long)c + 2ll * gridDim.x < (long long)nc;
        unsigned int next = 0u;
        if (tid == 0 && early) next = atomicAdd(&ctr[0], 1u);
        const long long u0 = (long long)(((unsigned long long)g.n_units * c) / nc);
        const long long u1 = (long long)(((unsigned long long)g.n_units * (c + 1)) / nc);
        acc |= or_units<U>(g, u0, u1);
        __syncthreads();
        if (tid == 0) s_chunk = (int)(early ? next : atomicAdd(&ctr[0], 1u));
        __syncthreads();
    }
    or_out(acc, out);
    if (tid == 0) {
        // Every block's claims are done before it takes this ticket.
        s_last = atomicAdd(&ctr[1], 1u) == gridDim.x - 1u ? 1u : 0u;
        if (s_last) {
            ctr[0] = 0u;
            ctr[1] = 0u;
        }
    }
}

}  // namespace

}  // namespace cube

using namespace cube;

extern "C" {

int cube_read_probe(const float *ptr, const int64_t *dims, int32_t nbins, uint32_t *dev_out,
                    void *stream)
{
    Box b;
    int rc = check_box(ptr, dims, &b);
    if (rc) return rc;
    if (nbins < 1 || nbins > CUBE_MAX_BINS)
        return fail(CUBE_EINVAL, "nbins=%d outside [1, %d]", nbins, CUBE_MAX_BINS);
    if (!dev_out) return fail(CUBE_EINVAL, "dev_out is NULL");
    if ((uintptr_t)dev_out % 4) return fail(CUBE_EINVAL, "dev_out is not 4-byte aligned");
    if (b.n == 0) return CUBE_OK;
    if ((rc = check_box_device(&b))) return rc;
    Plan p;
    if ((rc = make_plan(b, true, 1, nbins, &p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool dyn = p.chunks > 0;
    const void *k = dyn ? (p.unroll == 2 ? reinterpret_cast<const void *>(&k_probe_dyn<2>)
                                         : reinterpret_cast<const void *>(&k_probe_dyn<4>))
                        : (p.unroll == 2 ? reinterpret_cast<const void *>(&k_probe<2>)
                                         : reinterpret_cast<const void *>(&k_probe<4>));
    hipError_t e;
    if (p.lds > 64 * 1024 &&
        (e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds)) !=
            hipSuccess)
        return hip_fail(e, "probe LDS size");
    Geom g = p.g;
    unsigned int *out = dev_out;
    if (!dyn) {
        void *args[] = {&g, &out};
        e = hipLaunchKernel(k, dim3((unsigned)p.blocks), dim3((unsigned)p.threads), args, p.lds,
                            s);
        return e == hipSuccess ? CUBE_OK : hip_fail(e, "probe launch");
    }
    unsigned int *ctr = nullptr;
    if ((rc = stream_counter(s, &ctr))) return rc;
    int nc = p.chunks;
    void *args[] = {&g, &out, &ctr, &nc};
    e = hipLaunchKernel(k, dim3((unsigned)p.blocks), dim3((unsigned)p.threads), args, p.lds, s);
    if (e != hipSuccess) return hip_fail(e, "probe launch");
    return stream_used(s);
}

}  // extern "C"
