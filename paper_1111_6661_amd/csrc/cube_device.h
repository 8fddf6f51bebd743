// cube_device.h -- device code shared by the single-box and the batched
// kernels of the cube statistics library: the per-voxel step, the scan of a
// box's work units, the wavefront record (local stage), the LDS histogram
// flush and the FP64 merge of records (global stage).
//
// Per voxel:
//   * blank test (x != x), counted with a wavefront ballot on the scalar unit;
//   * min / max of the quieted value (v_min3/v_max3 order -0 before +0 and
//     skip quiet NaNs; a signalling NaN is quieted first);
//   * moments d = x - K and d^2 about a per-wavefront pivot K (the first
//     valid voxel the wavefront meets), summed in FP32 over a chunk of at most
//     two tiles and folded into a TwoSum-compensated lane accumulator
//     (Knuth's TwoSum);
//   * the histogram bin min(nbins-1, floor((x - lo) * scale)) in FP32 (two
//     rounded operations, then v_cvt_flr_i32_f32), counted in LDS
//     sub-histograms interleaved per lane; blank and out-of-range voxels go
//     to a dummy slot and are counted with ballots instead.
#pragma once

#include <math.h>

#include <type_traits>

#include "cube_internal.h"

namespace cube {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int MAX_WAVES = 16;   // 1024 threads per block at most

__device__ __forceinline__ int cvt_flr_i32(float u)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(u));
    return r;
}

__device__ __forceinline__ float qnan() { return __int_as_float(0x7fc00000); }

// s + c += x with the rounding error of s + x kept in c (TwoSum).
__device__ __forceinline__ void two_sum_acc(float &s, float &c, float x)
{
    const float t = s + x;
    const float bp = t - s;
    const float e = (s - (t - bp)) + (x - bp);
    s = t;
    c += e;
}

// (ah, al) += (bh, bl), double-float addition.
__device__ __forceinline__ void df_add(float &ah, float &al, float bh, float bl)
{
    const float s = ah + bh;
    const float bp = s - ah;
    float e = (ah - (s - bp)) + (bh - bp);
    e += al + bl;
    ah = s + e;
    al = e - (ah - s);
}

struct Lane {
    float mn, mx, s1, c1, s2, c2;
    float p1, p2;  // FP32 chunk sums not yet folded into (s1, c1), (s2, c2)
};

// Fold the pending FP32 chunk sums into the compensated lane accumulators
// (TwoSum).  Called after every second tile and at the end of every unit, so
// a chunk spans at most two tiles (32 voxels per lane) plus head and tail.
template <bool STATS, int ACC>
__device__ __forceinline__ void fold(Lane &L)
{
    if (STATS && ACC != CUBE_ACCUM_NAIVE32) {
        two_sum_acc(L.s1, L.c1, L.p1);
        two_sum_acc(L.s2, L.c2, L.p2);
        L.p1 = 0.f;
        L.p2 = 0.f;
    }
}

struct Wave {  // wavefront-uniform
    float K;
    int has_k;
    unsigned long long valid, ge, le;  // ballot counts: valid, x >= lo, x <= hi
};

// The histogram as one voxel sees it.  LDS layout: slot s of copy c is the
// word s * C + c (C = 1 << copies_log2 copies, interleaved so that lanes of
// one wavefront hitting the same bin hit different banks).  Slot 0 collects
// blank and out-of-range voxels (they are counted with ballots instead);
// slots 1..nbins are bins 0..nbins-1; slot nbins+1 collects the rounding
// case floor(u) == nbins and is added to bin nbins-1 at the flush (this is
// the min(nbins-1, .) of the bin rule).  The byte address of bin b for a
// lane is (b << shift) + base with base = (C + lane % C) * 4, so the dummy
// slot is b = -1, an inline constant.
//
// With a hot bin (HIST_HOT), lanes whose bin is the block's hot bin add
// nothing to LDS; out-of-range and blank lanes are masked off instead of
// going to the dummy slot.
struct Hist {
    float lo, hi, scale;
    int nbins, shift, base;
    int hot;  // HIST_HOT: the block's hot bin (0..nbins), or -2 for none
    unsigned int base_abs;  // HIST_HOT: base plus the LDS byte address of `lds`
    unsigned int *lds;
    unsigned long long *global;
};

// LDS word at byte address `addr` += 1 in the lanes of `m` only: the exec
// mask is narrowed around one ds_add_u32 and restored in the same asm block,
// so the step stays one basic block (a compiler branch per voxel splits the
// loop into small blocks and spills its lane masks).  The compiler does not
// count this LDS operation: whoever reads the histogram waits for it with
// lds_wait() first.
__device__ __forceinline__ void lds_add1_masked(unsigned int addr, unsigned long long m)
{
    unsigned long long saved;
    asm volatile(
        "s_and_saveexec_b64 %0, %1\n\t"
        "ds_add_u32 %2, %3\n\t"
        "s_or_b64 exec, exec, %0"
        : "=&s"(saved)
        : "s"(m), "v"(addr), "v"(1u)
        : "memory", "scc");
}

__device__ __forceinline__ void lds_wait()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// The byte address of an LDS pointer (the LDS aperture keeps the offset in
// the low 32 bits of a generic address).
__device__ __forceinline__ unsigned int lds_offset(const unsigned int *p)
{
    return (unsigned int)(size_t)(__attribute__((address_space(3))) const unsigned int *)p;
}

// m[lane] ? v : 0, and m[lane] ? v : -1 -- one v_cndmask_b32 reading a
// ballot mask directly, so a mask a ballot already produced is reused.
__device__ __forceinline__ float keep_where(float v, unsigned long long m)
{
    float r;
    asm("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(m));
    return r;
}
__device__ __forceinline__ int keep_or_minus1(int v, unsigned long long m)
{
    int r;
    asm("v_cndmask_b32_e64 %0, -1, %1, %2" : "=v"(r) : "v"(v), "s"(m));
    return r;
}

// One step over NV voxels per lane.  With a histogram, two compares decide
// everything: A = (x >= lo), B = (x <= hi) are both false for a NaN and,
// since lo <= hi, not both false otherwise, so valid = A|B, in-range = A&B,
// and below = valid - |A|, above = valid - |B| (scalar mask algebra and
// popcounts on the ballots).
template <bool STATS, int HIST, int ACC, int NV>
__device__ __forceinline__ void process(const float (&x)[NV], Lane &L, Wave &W,
                                        const Hist &H)
{
    if (STATS && ACC != CUBE_ACCUM_NAIVE32 && !W.has_k) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const unsigned long long m = __builtin_amdgcn_ballot_w64(x[j] == x[j]);
            if (m) {
                const int l = __builtin_ctzll(m);
                W.K = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[j]), l));
                W.has_k = 1;
                break;
            }
        }
    }
    // Ballot counts of this step in 32-bit scalars (at most 64 * NV each).
    unsigned int cvalid = 0, cge = 0, cle = 0;
    float t1 = L.p1, t2 = L.p2;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const float v = x[j];
        unsigned long long mvalid, inr = 0;
        const bool ge = v >= H.lo, le = v <= H.hi;
        if (HIST != HIST_NONE) {
            const unsigned long long mge = __builtin_amdgcn_ballot_w64(ge);
            const unsigned long long mle = __builtin_amdgcn_ballot_w64(le);
            mvalid = mge | mle;
            inr = mge & mle;
            cge += __popcll(mge);
            cle += __popcll(mle);
        } else {
            mvalid = __builtin_amdgcn_ballot_w64(v == v);
        }
        cvalid += __popcll(mvalid);
        if (STATS) {
            const float q = __builtin_canonicalizef(v);
            L.mn = fminf(L.mn, q);
            L.mx = fmaxf(L.mx, q);
            if (ACC == CUBE_ACCUM_NAIVE32) {
                const float d = keep_where(v, mvalid);
                L.s1 += d;
                L.s2 = __fmaf_rn(d, d, L.s2);
            } else {
                const float d = keep_where(__fsub_rn(v, W.K), mvalid);
                t1 += d;
                t2 = __fmaf_rn(d, d, t2);
            }
        }
        if (HIST != HIST_NONE) {
            const float u = __fmul_rn(__fsub_rn(v, H.lo), H.scale);
            if (HIST == HIST_LDS) {
                const int b = keep_or_minus1(cvt_flr_i32(u), inr);
                atomicAdd((unsigned int *)((char *)H.lds + ((b << H.shift) + H.base)), 1u);
            } else if (HIST == HIST_HOT) {
                // Only in-range lanes off the hot bin touch LDS.
                const int b = cvt_flr_i32(u);
                const unsigned long long off_hot = __builtin_amdgcn_ballot_w64(b != H.hot);
                lds_add1_masked((unsigned int)((b << H.shift) + H.base_abs), inr & off_hot);
            } else {
                const int b = min(cvt_flr_i32(u), H.nbins - 1);
                if ((inr >> (threadIdx.x & 63)) & 1ull) atomicAdd(&H.global[b], 1ull);
            }
        }
    }
    // Keep the step counts 32-bit (the compiler would otherwise widen every
    // per-voxel add to 64 bits).
    asm("" : "+s"(cvalid), "+s"(cge), "+s"(cle));
    W.valid += cvalid;
    W.ge += cge;
    W.le += cle;
    if (STATS && ACC != CUBE_ACCUM_NAIVE32) {
        L.p1 = t1;
        L.p2 = t2;
    }
}

// Pairwise merge of (n, mean, m2) summaries (Chan, Golub & LeVeque).
template <typename T>
__device__ __forceinline__ void chan_merge(double &n, T &mean, T &m2, double nb, T mb, T m2b)
{
    if (nb == 0.0) return;
    if (n == 0.0) {
        n = nb;
        mean = mb;
        m2 = m2b;
        return;
    }
    const double nt = n + nb;
    const T d = mb - mean;
    mean = mean + d * (T)(nb / nt);
    m2 = m2 + m2b + d * d * (T)(n * nb / nt);
    n = nt;
}

template <typename T>
struct Summary {
    double n;
    T mean, m2;
    float mn, mx;
    unsigned long long nv, below, above;
};

template <typename T>
__device__ __forceinline__ void summary_merge(Summary<T> &a, const Summary<T> &b)
{
    chan_merge<T>(a.n, a.mean, a.m2, b.n, b.mean, b.m2);
    a.mn = fminf(a.mn, b.mn);
    a.mx = fmaxf(a.mx, b.mx);
    a.nv += b.nv;
    a.below += b.below;
    a.above += b.above;
}

template <typename T>
__device__ __forceinline__ Summary<T> shfl_xor_summary(const Summary<T> &s, int off)
{
    Summary<T> o;
    o.n = __shfl_xor(s.n, off);
    o.mean = __shfl_xor(s.mean, off);
    o.m2 = __shfl_xor(s.m2, off);
    o.mn = __shfl_xor(s.mn, off);
    o.mx = __shfl_xor(s.mx, off);
    o.nv = __shfl_xor(s.nv, off);
    o.below = __shfl_xor(s.below, off);
    o.above = __shfl_xor(s.above, off);
    return o;
}

// The (count, mean, m2) of one wavefront record: its pivoted sums
// S1 = sum(x - K), S2 = sum((x - K)^2) give mean = K + S1/n and
// m2 = S2 - S1^2/n (clamped at 0).
template <typename T, int ACC>
__device__ __forceinline__ void moments_of(const WaveRec &w, T &mb, T &m2b)
{
    const double nb = (double)w.n_valid;
    if (ACC == CUBE_ACCUM_NAIVE32) {
        const T S1 = (T)w.s1h, S2 = (T)w.s2h, n = (T)nb;
        mb = S1 / n;
        m2b = S2 - S1 * S1 / n;
    } else {
        const T S1 = (T)w.s1h + (T)w.s1l;
        const T S2 = (T)w.s2h + (T)w.s2l;
        mb = (T)w.K + S1 / (T)nb;
        m2b = S2 - S1 * S1 / (T)nb;
    }
    if (m2b < (T)0) m2b = (T)0;
}

// A chunk record already holds its mean and m2.
template <typename T, int ACC>
__device__ __forceinline__ void moments_of(const ChunkRec &c, T &mb, T &m2b)
{
    mb = (T)c.mean;
    m2b = (T)c.m2;
}

// The global stage: every thread folds a fixed slice of the records (wave
// records, or chunk records in chunk order) in order, then a fixed xor-tree
// inside each wavefront, then the wavefront summaries in order.
// Deterministic for a given record count.
template <typename T, int ACC, typename R = WaveRec>
__device__ Summary<T> merge_records(const R *recs, int n_recs)
{
    const int tid = threadIdx.x, B = blockDim.x;
    const int r0 = (int)(((long long)n_recs * tid) / B);
    const int r1 = (int)(((long long)n_recs * (tid + 1)) / B);
    Summary<T> s = {0.0, (T)0, (T)0, INFINITY, -INFINITY, 0ull, 0ull, 0ull};
    for (int r = r0; r < r1; ++r) {
        const R w = recs[r];
        s.below += w.below;
        s.above += w.above;
        if (w.n_valid == 0) continue;
        s.nv += w.n_valid;
        s.mn = fminf(s.mn, w.mn);
        s.mx = fmaxf(s.mx, w.mx);
        T mb, m2b;
        moments_of<T, ACC>(w, mb, m2b);
        chan_merge<T>(s.n, s.mean, s.m2, (double)w.n_valid, mb, m2b);
    }
    for (int off = 1; off < 64; off <<= 1) {
        Summary<T> o = shfl_xor_summary(s, off);
        // Fixed pairing: the lower lane of each pair is the left operand.
        if ((threadIdx.x & off) == 0) {
            summary_merge(s, o);
        } else {
            summary_merge(o, s);
            s = o;
        }
    }
    __shared__ Summary<T> ws[MAX_WAVES];
    const int lane = tid & 63, wid = tid >> 6, nw = B >> 6;
    if (lane == 0) ws[wid] = s;
    __syncthreads();
    Summary<T> t = ws[0];
    for (int w = 1; w < nw; ++w) summary_merge(t, ws[w]);
    return t;
}

// A fixed-order sum over the block of one double and the counts and
// extrema that travel with it: an xor-tree inside each wavefront (the lower
// lane of each pair on the left), then the wavefront results in order.
// Every thread gets the result.
struct BlockSums {
    double s;
    unsigned long long nv, below, above;
    float mn, mx;
};

__device__ __forceinline__ BlockSums block_sums(BlockSums v)
{
    for (int off = 1; off < 64; off <<= 1) {
        const double os = __shfl_xor(v.s, off);
        const unsigned long long onv = __shfl_xor(v.nv, off);
        const unsigned long long ob = __shfl_xor(v.below, off);
        const unsigned long long oa = __shfl_xor(v.above, off);
        const float omn = __shfl_xor(v.mn, off), omx = __shfl_xor(v.mx, off);
        v.s = (threadIdx.x & off) == 0 ? v.s + os : os + v.s;
        v.nv += onv;
        v.below += ob;
        v.above += oa;
        v.mn = fminf(v.mn, omn);
        v.mx = fmaxf(v.mx, omx);
    }
    __shared__ BlockSums ws[MAX_WAVES];
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();  // a previous call's readers are done with ws
    if ((threadIdx.x & 63) == 0) ws[wid] = v;
    __syncthreads();
    BlockSums t = ws[0];
    for (int w = 1; w < nw; ++w) {
        t.s += ws[w].s;
        t.nv += ws[w].nv;
        t.below += ws[w].below;
        t.above += ws[w].above;
        t.mn = fminf(t.mn, ws[w].mn);
        t.mx = fmaxf(t.mx, ws[w].mx);
    }
    return t;
}

// The two terms each record adds to the two sweeps of the FP64 global
// stage below: its sum of x, and its sum of (x - mean)^2 about the global
// mean.  A chunk record holds (n, mean_c, m2_c): n * mean_c and
// m2_c + n * (mean_c - mean)^2.  A wavefront record holds the pivoted sums
// S1 = sum(x - K), S2 = sum((x - K)^2): n * K + S1 and, with d = K - mean,
// sum((x - K) + d)^2 = S2 + 2 d S1 + n d^2.  Both forms are exact identities;
// neither divides.
__device__ __forceinline__ double sweep1_term(const ChunkRec &c)
{
    return (double)c.n_valid * c.mean;
}
__device__ __forceinline__ double sweep2_term(const ChunkRec &c, double mean)
{
    const double d = c.mean - mean;
    return c.m2 + (double)c.n_valid * d * d;
}
__device__ __forceinline__ double sweep1_term(const WaveRec &w)
{
    return (double)w.n_valid * (double)w.K + ((double)w.s1h + (double)w.s1l);
}
__device__ __forceinline__ double sweep2_term(const WaveRec &w, double mean)
{
    const double d = (double)w.K - mean;
    const double S1 = (double)w.s1h + (double)w.s1l;
    const double S2 = (double)w.s2h + (double)w.s2l;
    return S2 + 2.0 * d * S1 + (double)w.n_valid * d * d;
}

// The FP64 global stage in two sweeps over the records, with no division
// per record: the counts and the records' sums of x give the mean, then the
// records' sums of (x - mean)^2 give M2 -- the exact combination that the
// pairwise update of Chan, Golub & LeVeque applies two at a time.  Thread t
// takes records t, t + B, ... (coalesced loads, four in flight), then
// block_sums fixes the rest of the order.  Deterministic for a given record
// count and block size.
template <typename R>
__device__ Summary<double> merge_two_sweep(const R *recs, int n_recs)
{
    const int tid = threadIdx.x, B = blockDim.x;
    BlockSums a = {0.0, 0ull, 0ull, 0ull, INFINITY, -INFINITY};
    auto take1 = [&](const R &c) {
        a.below += c.below;
        a.above += c.above;
        if (c.n_valid == 0) return;
        a.nv += c.n_valid;
        a.mn = fminf(a.mn, c.mn);
        a.mx = fmaxf(a.mx, c.mx);
        a.s += sweep1_term(c);
    };
    int r = tid;
    for (; r + 3 * B < n_recs; r += 4 * B) {
        R c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = recs[r + k * B];
#pragma unroll
        for (int k = 0; k < 4; ++k) take1(c[k]);
    }
    for (; r < n_recs; r += B) take1(recs[r]);
    const BlockSums t = block_sums(a);
    const double mean = t.nv ? t.s / (double)t.nv : 0.0;
    BlockSums m = {0.0, 0ull, 0ull, 0ull, INFINITY, -INFINITY};
    auto take2 = [&](const R &c) {
        if (c.n_valid) m.s += sweep2_term(c, mean);
    };
    for (r = tid; r + 3 * B < n_recs; r += 4 * B) {
        R c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = recs[r + k * B];
#pragma unroll
        for (int k = 0; k < 4; ++k) take2(c[k]);
    }
    for (; r < n_recs; r += B) take2(recs[r]);
    const BlockSums u = block_sums(m);
    Summary<double> S;
    S.n = (double)t.nv;
    S.mean = mean;
    S.m2 = u.s;
    S.mn = t.mn;
    S.mx = t.mx;
    S.nv = t.nv;
    S.below = t.below;
    S.above = t.above;
    return S;
}

// One tile: U float4 loads per lane, lane stride B (a wavefront reads 1 KB
// per load); a uniform base plus fixed per-lane 32-bit byte offsets.
template <int U>
__device__ __forceinline__ void load_tile(f4 (&v)[U], const f4 *q4, long long off, int B, int tid)
{
    const char *base = (const char *)(q4 + off);
#pragma unroll
    for (int k = 0; k < U; ++k)
        v[k] = __builtin_nontemporal_load((const f4 *)(base + (unsigned int)((k * B + tid) * 16)));
}

template <bool STATS, int HIST, int ACC, int U>
__device__ __forceinline__ void process_tile(const f4 (&v)[U], Lane &L, Wave &W, const Hist &H)
{
    float xv[4 * U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        xv[4 * k + 0] = v[k].x;
        xv[4 * k + 1] = v[k].y;
        xv[4 * k + 2] = v[k].z;
        xv[4 * k + 3] = v[k].w;
    }
    process<STATS, HIST, ACC, 4 * U>(xv, L, W, H);
}

// Histogram context of a pass over the valid range r (an invalid range is
// handled by the caller with a pass without histogram).
__device__ __forceinline__ void hist_setup(Hist &H, const HistRange &r, int nbins,
                                           int copies_log2, unsigned int *lds,
                                           unsigned long long *acc)
{
    const int lane = threadIdx.x & 63;
    const int C = 1 << copies_log2;
    H.hot = -2;
    H.nbins = nbins;
    H.shift = copies_log2 + 2;
    H.base = (C + (lane & (C - 1))) * 4;
    H.base_abs = (unsigned int)H.base + lds_offset(lds);
    H.lds = lds;
    H.global = acc;
    H.lo = r.lo;
    H.hi = r.hi;
    H.scale = r.scale;
}

// Zero the LDS sub-histograms (nbins + 2 slots per copy); ends with a barrier.
__device__ __forceinline__ void lds_zero(unsigned int *lds, int nbins, int copies_log2)
{
    const int words = (nbins + 2) << copies_log2;
    for (int i = threadIdx.x; i < words; i += blockDim.x) lds[i] = 0u;
    __syncthreads();
}

// The "last block merges" ticket.  Called by every thread of the block after
// its writes.  After a barrier, thread 0 issues one agent-scope release fence
// (fences are cumulative: it covers every thread's writes ordered before it
// by the barrier; on gfx950 it writes back the L2), takes a ticket and, if it
// is the last of `total`, one agent-scope acquire fence (an L2 and L1
// invalidate) before the barrier that lets the block read the others' writes.
// A full __threadfence() is both, and one in every thread costs a write-back
// per wavefront.  Returns the same answer to every thread.
__device__ __forceinline__ bool last_to_arrive(unsigned int *ticket, unsigned int total,
                                               unsigned int *s_shared)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const bool last = atomicAdd(ticket, 1u) == total - 1u;
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_shared = last ? 1u : 0u;
    }
    __syncthreads();
    return *s_shared != 0u;
}

// The same election without the L2 write-back of the release fence, for a
// block whose every write that the last block reads is an agent-scope atomic
// store (written through the XCD's L2 to the device's point of coherence) or
// an agent-scope atomic read-modify-write (performed there).  Each wavefront
// waits for its own such writes to complete before the barrier, so all of
// them are performed at device scope before thread 0 takes the ticket; the
// last block then acquires (invalidates its L2) before it reads.  The release
// fence's buffer_wbl2 would only add the write-back of plain stores, of
// which there are none here; it stalls a block for several microseconds per
// call, which the batched launch pays at every tile.
__device__ __forceinline__ bool last_to_arrive_wt(unsigned int *ticket, unsigned int total,
                                                  unsigned int *s_shared)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool last = atomicAdd(ticket, 1u) == total - 1u;
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_shared = last ? 1u : 0u;
    }
    __syncthreads();
    return *s_shared != 0u;
}

// Scan the work units [u0, u1) of a box (segments of rows, see Geom).
template <bool STATS, int HIST, int ACC, int U>
__device__ __forceinline__ void scan_units(const Geom &g, long long u0, long long u1, Lane &L,
                                           Wave &W, const Hist &H)
{
    if (u0 >= u1) return;
    const int tid = threadIdx.x, B = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6;
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
            // Head and tail voxels: lanes [0, h) and [h, h + t).
            long long idx = lane < h ? lane : h + 4 * n4 + (lane - h);
            const bool have = lane < h + t;
            idx = have ? idx : 0;
            float xv[1];
            const float v = q[idx];
            xv[0] = have ? v : qnan();
            process<STATS, HIST, ACC, 1>(xv, L, W, H);
        }
        const f4 *q4 = (const f4 *)(q + h);
        // Full tiles, software-pipelined: the next tile's loads are in
        // flight while the current tile is processed.
        const long long T = (long long)B * U;
        const long long ntiles = n4 / T;
        if (ntiles > 0) {
            f4 va[U], vb[U];
            load_tile<U>(va, q4, 0, B, tid);
            long long k = 0;
            while (true) {
                if (k + 1 < ntiles) load_tile<U>(vb, q4, (k + 1) * T, B, tid);
                process_tile<STATS, HIST, ACC, U>(va, L, W, H);
                if (++k == ntiles) break;
                if (k + 1 < ntiles) load_tile<U>(va, q4, (k + 1) * T, B, tid);
                process_tile<STATS, HIST, ACC, U>(vb, L, W, H);
                fold<STATS, ACC>(L);
                if (++k == ntiles) break;
            }
        }
        for (long long i0 = ntiles * T; i0 < n4; i0 += B) {
            const long long i = i0 + tid;
            const bool have = i < n4;
            const f4 v = __builtin_nontemporal_load(q4 + (have ? i : n4 - 1));
            float xv[4];
            xv[0] = have ? v.x : qnan();
            xv[1] = have ? v.y : qnan();
            xv[2] = have ? v.z : qnan();
            xv[3] = have ? v.w : qnan();
            process<STATS, HIST, ACC, 4>(xv, L, W, H);
        }
        fold<STATS, ACC>(L);
        if (++s == g.segs) {
            s = 0;
            if (++y == g.ny) {
                y = 0;
                ++z;
            }
        }
    }
}

// Local stage: reduce the lanes of the calling wavefront into one record
// (written by lane 0).
// With WT (write-through) lane 0 writes the record as sixteen agent-scope
// atomic stores, which gfx950 writes through its XCD's L2 (see
// last_to_arrive_wt); otherwise as plain stores.
template <bool STATS, int ACC, bool WT = false>
__device__ __forceinline__ void write_wave_record(const Lane &L, const Wave &W, WaveRec *dst)
{
    float mn = L.mn, mx = L.mx, s1h = L.s1, s1l = L.c1, s2h = L.s2, s2l = L.c2;
    if (STATS) {
        for (int off = 32; off > 0; off >>= 1) {
            mn = fminf(mn, __shfl_xor(mn, off));
            mx = fmaxf(mx, __shfl_xor(mx, off));
            const float o1h = __shfl_xor(s1h, off), o1l = __shfl_xor(s1l, off);
            const float o2h = __shfl_xor(s2h, off), o2l = __shfl_xor(s2l, off);
            if (ACC == CUBE_ACCUM_NAIVE32) {
                s1h += o1h;
                s2h += o2h;
            } else {
                df_add(s1h, s1l, o1h, o1l);
                df_add(s2h, s2l, o2h, o2l);
            }
        }
    }
    if ((threadIdx.x & 63) == 0) {
        WaveRec r;
        r.n_valid = W.valid;
        r.below = W.valid - W.ge;
        r.above = W.valid - W.le;
        r.K = W.K;
        r.s1h = s1h;
        r.s1l = s1l;
        r.s2h = s2h;
        r.s2l = s2l;
        r.mn = mn;
        r.mx = mx;
        r.pad = 0.f;
        r.pad2 = 0ull;
        if (WT) {
            const unsigned int *w = reinterpret_cast<const unsigned int *>(&r);
            unsigned int *d = reinterpret_cast<unsigned int *>(dst);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                __hip_atomic_store(d + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            *dst = r;
        }
    }
}

// The record of one chunk of a dynamic partition, formed by the first
// wavefront from the block's wavefront records of that chunk (`parts`, in
// LDS, `nw` of them): lane i takes record i, the lanes are merged in FP64 by
// a fixed xor-tree (the lower lane of each pair on the left), and lane 0
// writes the result.  Without STATS only the counts are kept.
template <bool STATS>
__device__ __forceinline__ void write_chunk_record(const WaveRec *parts, int nw, ChunkRec *dst)
{
    const int lane = threadIdx.x & 63;
    Summary<double> s = {0.0, 0.0, 0.0, INFINITY, -INFINITY, 0ull, 0ull, 0ull};
    if (lane < nw) {
        const WaveRec w = parts[lane];
        s.below = w.below;
        s.above = w.above;
        s.nv = w.n_valid;
        if (STATS && w.n_valid) {
            s.n = (double)w.n_valid;
            s.mn = w.mn;
            s.mx = w.mx;
            moments_of<double, CUBE_ACCUM_FP64MERGE>(w, s.mean, s.m2);
        }
    }
    for (int off = 1; off < MAX_WAVES; off <<= 1) {
        if (STATS) {
            Summary<double> o = shfl_xor_summary(s, off);
            if ((lane & off) == 0) {
                summary_merge(s, o);
            } else {
                summary_merge(o, s);
                s = o;
            }
        } else {
            s.nv += __shfl_xor(s.nv, off);
            s.below += __shfl_xor(s.below, off);
            s.above += __shfl_xor(s.above, off);
        }
    }
    if (lane == 0) {
        ChunkRec c;
        c.mean = s.mean;
        c.m2 = s.m2;
        c.mn = s.mn;
        c.mx = s.mx;
        c.pad0 = c.pad1 = 0u;
        c.n_valid = s.nv;
        c.below = s.below;
        c.above = s.above;
        c.pad2 = 0ull;
        *dst = c;
    }
}

// Add the block's LDS sub-histograms into the global accumulators (one
// atomic per non-empty bin).  Starts with a barrier.
__device__ __forceinline__ void hist_flush(const unsigned int *lds, int nbins, int copies_log2,
                                           unsigned long long *acc)
{
    __syncthreads();
    const int C = 1 << copies_log2;
    // Each thread starts at its own copy (c + tid) so that the threads of a
    // wavefront read different banks at every step.
    const int rot = threadIdx.x;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        unsigned int sum = 0;
        for (int c = 0; c < C; ++c) sum += lds[((b + 1) << copies_log2) + ((c + rot) & (C - 1))];
        if (b == nbins - 1)  // floor(u) == nbins belongs to the last bin
            for (int c = 0; c < C; ++c) sum += lds[((nbins + 1) << copies_log2) + c];
        if (sum) atomicAdd(&acc[b], (unsigned long long)sum);
    }
}

// The hot bin of a block (HIST_HOT), chosen by its first wavefront before the
// scan: the bin of the first in-range voxel among the first 64 of the block's
// first work unit, computed with the same FP32 operations as every voxel's
// bin (any value is correct; a likely one saves LDS atomics).  -2: none.
__device__ __forceinline__ int hot_bin_pick(const Geom &g, long long u0, long long u1,
                                            const Hist &H)
{
    if (u0 >= u1) return -2;
    const int lane = threadIdx.x & 63;
    const long long row = u0 / g.segs;
    const long long sg = u0 - row * g.segs;
    const long long y = row % g.ny, z = row / g.ny;
    const long long c0 = sg * g.seg_len;
    const long long len = min(g.seg_len, g.row_len - c0);
    const float *q = g.ptr + y * g.sy + z * g.sz + c0;
    const float v = lane < len ? q[lane] : qnan();
    const int b = cvt_flr_i32(__fmul_rn(__fsub_rn(v, H.lo), H.scale));
    const unsigned long long m = __builtin_amdgcn_ballot_w64(v >= H.lo && v <= H.hi);
    if (!m) return -2;
    return __builtin_amdgcn_readlane(b, __builtin_ctzll(m));
}

// The flush of a hot-bin histogram: every other bin as in hist_flush, then
// the hot bin's count, which is the block's in-range count (`s_inr`, summed
// from the wavefronts' ballot counts) minus everything the block added to
// LDS (`s_tot`, zeroed before the scan).  Starts with a barrier.
__device__ __forceinline__ void hist_flush_hot(const unsigned int *lds, int nbins,
                                               int copies_log2, unsigned long long *acc,
                                               int hot, const unsigned int *s_inr,
                                               unsigned int *s_tot)
{
    lds_wait();  // the masked LDS adds of this wavefront
    __syncthreads();
    const int C = 1 << copies_log2;
    const int rot = threadIdx.x;
    unsigned int mine = 0;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        unsigned int sum = 0;
        for (int c = 0; c < C; ++c) sum += lds[((b + 1) << copies_log2) + ((c + rot) & (C - 1))];
        if (b == nbins - 1)  // floor(u) == nbins belongs to the last bin
            for (int c = 0; c < C; ++c) sum += lds[((nbins + 1) << copies_log2) + c];
        mine += sum;
        if (sum) atomicAdd(&acc[b], (unsigned long long)sum);
    }
    if (mine) atomicAdd(s_tot, mine);
    __syncthreads();
    if (threadIdx.x == 0 && hot >= 0) {
        const unsigned int n_hot = *s_inr - *s_tot;
        if (n_hot) atomicAdd(&acc[hot < nbins ? hot : nbins - 1], (unsigned long long)n_hot);
    }
}

// The in-range count of the calling wavefront (ballots: x >= lo, x <= hi and
// valid = either), added to the block's LDS counter by lane 0.
__device__ __forceinline__ void add_in_range(const Wave &W, unsigned int *s_inr)
{
    if ((threadIdx.x & 63) == 0)
        atomicAdd(s_inr, (unsigned int)(W.ge + W.le - W.valid));
}

// The [min, max] histogram range with its FP32 scale, formed from the data
// extrema exactly as the host forms a given range: ok = 1 valid, 0 invalid
// (infinite extrema, or a width or scale that overflows), 2 no valid voxel.
__device__ __forceinline__ HistRange range_of_extrema(float fmn, float fmx, unsigned long long nv,
                                                      int nbins)
{
    HistRange r = {qnan(), qnan(), 0.f, 2};
    if (nv == 0) return r;
    r.ok = 0;
    if (isfinite(fmn) && isfinite(fmx)) {
        const float w = __fsub_rn(fmx, fmn);
        if (isfinite(w)) {
            const float sc = w == 0.f ? 0.f : __fdiv_rn((float)nbins, w);
            if (isfinite(sc)) {
                r.lo = fmn;
                r.hi = fmx;
                r.scale = sc;
                r.ok = 1;
            }
        }
    }
    return r;
}

// Moments over the extended reals.  An infinite voxel is a valid value and
// always one of the extrema, so the exact min and max show whether any are
// present, at no cost per voxel: +Inf alone makes the mean +Inf, -Inf alone
// -Inf, both NaN (Inf - Inf); and since the deviation of an infinite voxel
// from such a mean is not finite, m2 and std are NaN.  Without infinities
// the merged finite moments stand.
__device__ __forceinline__ void extended_real_moments(cube_stats_t &o)
{
    const bool pinf = o.max == INFINITY, ninf = o.min == -INFINITY;
    if (!pinf && !ninf) return;
    o.mean = (pinf && ninf) ? (double)qnan() : (pinf ? (double)INFINITY : -(double)INFINITY);
    o.m2 = o.std = (double)qnan();
}

// The global stage of a stats pass: merge `n_recs` records (all threads of
// the block call it), then thread 0 writes the result and, when `range_out`
// is given, the [min, max] histogram range with its FP32 scale.  Returns the
// total valid / below / above counts to every thread.
template <int ACC, typename R = WaveRec>
__device__ void finish_stats(const R *recs, int n_recs, int accum_mode,
                             unsigned long long n_total, cube_stats_t *out,
                             HistRange *range_out, int nbins, unsigned long long &nv,
                             unsigned long long &below, unsigned long long &above)
{
    float fmn, fmx;
    double mean, m2;
    if (accum_mode == CUBE_ACCUM_FP64MERGE) {
        // Pivoted wavefront records (FP64MERGE partials) and chunk records
        // take the two-sweep merge; the naive partials keep the pairwise one.
        Summary<double> S;
        if constexpr (std::is_same<R, ChunkRec>::value || ACC == CUBE_ACCUM_FP64MERGE)
            S = merge_two_sweep<R>(recs, n_recs);
        else
            S = merge_records<double, ACC, R>(recs, n_recs);
        nv = S.nv; below = S.below; above = S.above;
        fmn = S.mn; fmx = S.mx; mean = S.mean; m2 = S.m2;
    } else {
        const Summary<float> S = merge_records<float, ACC, R>(recs, n_recs);
        nv = S.nv; below = S.below; above = S.above;
        fmn = S.mn; fmx = S.mx; mean = (double)S.mean; m2 = (double)S.m2;
    }
    if (threadIdx.x != 0) return;
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
        o.min = fmn;
        o.max = fmx;
        o.mean = mean;
        o.m2 = m2 < 0.0 ? 0.0 : m2;
        o.std = accum_mode == CUBE_ACCUM_FP64MERGE ? sqrt(o.m2 / (double)nv)
                                                   : (double)sqrtf((float)o.m2 / (float)nv);
        extended_real_moments(o);
    }
    if (range_out) {
        const HistRange r = range_of_extrema(fmn, fmx, nv, nbins);
        if (r.ok == 0) o.flags |= CUBE_HIST_BAD_RANGE;
        *range_out = r;
    }
    *out = o;
}

// Copy the global accumulators to the caller's counts (or, with `add`, add
// them to the counts already there) and return them to zero; thread 0 writes
// below / above / NaN.
__device__ __forceinline__ void finish_hist(unsigned long long *acc, unsigned long long *counts,
                                            int nbins, bool on, unsigned long long below,
                                            unsigned long long above, unsigned long long n_nan,
                                            bool add = false)
{
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        counts[b] = (add ? counts[b] : 0ull) + acc[b];
        acc[b] = 0ull;
    }
    if (threadIdx.x == 0) {
        counts[nbins] = (add ? counts[nbins] : 0ull) + (on ? below : 0ull);
        counts[nbins + 1] = (add ? counts[nbins + 1] : 0ull) + (on ? above : 0ull);
        counts[nbins + 2] = (add ? counts[nbins + 2] : 0ull) + n_nan;
    }
}

}  // namespace cube
