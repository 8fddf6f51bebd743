// cube_kernels.hip -- the single-box pass of the cube statistics library.
//
// k_pass streams one box once (the device code is in cube_device.h): each
// block scans a contiguous range of work units, reduces its wavefronts into
// records (the local stage of the paper's two-stage gather, Section 2),
// flushes its LDS histogram with one 64-bit atomic per non-empty bin, and the
// last block to finish (a ticket counter) merges every record in a fixed
// order in FP64 (the global stage) and writes the results.  Results are
// deterministic for a given launch shape.  k_pass_dyn (below) is the same
// pass with the box handed out in chunks at run time.
#include "cube_device.h"

namespace cube {

template <bool STATS, int HIST, int ACC, int U>
__global__ void __launch_bounds__(1024) k_pass(PassArgs a)
{
    extern __shared__ unsigned int lds[];
    __shared__ unsigned int s_last;
    __shared__ unsigned int s_inr, s_tot;  // HIST_HOT: in-range and LDS-counted voxels
    __shared__ int s_hot;
    const int tid = threadIdx.x;
    const int wid = tid >> 6, nw = blockDim.x >> 6;

    Hist H;
    const HistRange r0 = {0.f, 0.f, 0.f, 0};
    const HistRange hr = HIST != HIST_NONE ? (a.dev_range ? *a.dev_range : a.range) : r0;
    const bool hist_on = HIST != HIST_NONE && hr.ok == 1;
    hist_setup(H, hr, a.nbins, a.copies_log2, lds, a.hist_acc);

    const Geom &g = a.g;
    const unsigned long long G = gridDim.x;
    const long long u0 = (long long)(((unsigned long long)g.n_units * blockIdx.x) / G);
    const long long u1 = (long long)(((unsigned long long)g.n_units * (blockIdx.x + 1)) / G);
    if (HIST == HIST_HOT) {
        // The hot bin and the two counters, published by lds_zero's barrier.
        if (wid == 0) {
            const int h = hist_on ? hot_bin_pick(g, u0, u1, H) : -2;
            if (tid == 0) {
                s_hot = h;
                s_inr = 0u;
                s_tot = 0u;
            }
        }
    }
    if (HIST == HIST_LDS || HIST == HIST_HOT) lds_zero(lds, a.nbins, a.copies_log2);
    if (HIST == HIST_HOT) H.hot = s_hot;

    Lane L = {INFINITY, -INFINITY, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    Wave W = {0.f, ACC == CUBE_ACCUM_NAIVE32 ? 1 : 0, 0ull, 0ull, 0ull};

    if (HIST == HIST_NONE || hist_on)
        scan_units<STATS, HIST, ACC, U>(g, u0, u1, L, W, H);
    else  // an invalid range bins nothing: count valid voxels only
        scan_units<STATS, HIST_NONE, ACC, U>(g, u0, u1, L, W, H);

    write_wave_record<STATS, ACC>(L, W, &a.recs[(long long)blockIdx.x * nw + wid]);
    if (HIST == HIST_LDS) hist_flush(lds, a.nbins, a.copies_log2, a.hist_acc);
    if (HIST == HIST_HOT) {
        if (hist_on) add_in_range(W, &s_inr);
        hist_flush_hot(lds, a.nbins, a.copies_log2, a.hist_acc, H.hot, &s_inr, &s_tot);
    }

    // Ticket: the last block to arrive performs the global stage.  One
    // release fence per block, not per thread: a fence in every thread costs
    // a write-back of the L2 per wavefront (measured: about a tenth of the
    // pass).
    if (!last_to_arrive(a.ticket, gridDim.x, &s_last)) return;

    const int n_recs = (int)gridDim.x * nw;
    unsigned long long nv, below, above;
    if (STATS) {
        finish_stats<ACC>(a.recs, n_recs, a.accum_mode, g.n_total, a.out,
                          a.want_range ? a.out_range : nullptr, a.nbins, nv, below, above);
    } else {
        const Summary<float> S = merge_records<float, CUBE_ACCUM_KAHAN32>(a.recs, n_recs);
        nv = S.nv;
        below = S.below;
        above = S.above;
    }
    if (HIST != HIST_NONE)
        finish_hist(a.hist_acc, a.counts, a.nbins, hist_on, below, above, g.n_total - nv,
                    a.accumulate != 0);
    if (tid == 0) *a.ticket = 0u;
}

// k_pass_dyn is the same pass with a dynamic partition: the box is cut into
// a.n_chunks chunks of consecutive work units, and each block claims the
// next chunk from a counter as it finishes one (blocks on faster parts of
// the chip take more chunks; a static partition ends when its slowest block
// does).  Every chunk gets one record, its wavefront records merged in FP64,
// and the last block merges the chunk records in chunk order, so results
// depend on the chunk count and the block shape (threads, loads per tile)
// but not on the grid or on which block took which chunk.  The LDS
// histogram is kept over all of a block's chunks and flushed once.  The
// moments are accumulated as in CUBE_ACCUM_FP64MERGE (the planner uses this
// pass for that mode only), without the hot-bin histogram form.
template <bool STATS, int HIST, int U>
__global__ void __launch_bounds__(1024) k_pass_dyn(PassArgs a)
{
    extern __shared__ unsigned int lds[];
    __shared__ unsigned int s_last;
    __shared__ int s_chunk;
    __shared__ int s_ids[MAX_WAVES];  // the chunks whose parts the ring holds
    const int tid = threadIdx.x;
    const int wid = tid >> 6, nw = blockDim.x >> 6;
    constexpr int ACC = CUBE_ACCUM_FP64MERGE;
    // The ring of wavefront records (dynamic LDS after the histogram): nw
    // chunks of nw records each.
    WaveRec *ring = reinterpret_cast<WaveRec *>(
        lds + dyn_ring_offset_words(HIST == HIST_LDS, a.nbins, a.copies_log2));

    Hist H;
    const HistRange r0 = {0.f, 0.f, 0.f, 0};
    const HistRange hr = HIST != HIST_NONE ? (a.dev_range ? *a.dev_range : a.range) : r0;
    const bool hist_on = HIST != HIST_NONE && hr.ok == 1;
    hist_setup(H, hr, a.nbins, a.copies_log2, lds, a.hist_acc);

    const Geom &g = a.g;
    const int nc = a.n_chunks;
    unsigned int *ctr = a.ticket + CHUNK_CTR_WORD;
    // A chunk spans at most this many voxels (whole units of seg_len floats).
    const long long chunk_max =
        (long long)((g.n_units + (unsigned long long)nc - 1) / (unsigned long long)nc) * g.seg_len;
    if (tid == 0) s_chunk = (int)atomicAdd(ctr, 1u);
    if (HIST == HIST_LDS) lds_zero(lds, a.nbins, a.copies_log2);  // ends with a barrier
    else __syncthreads();

    long long since_flush = 0;  // voxels counted in LDS since it was last zeroed
    int filled = 0;             // chunks in the ring (uniform)
    while (true) {
        const int c = s_chunk;
        if (c >= nc) break;
        // Claim the next chunk now, unless the list is near its end (a block
        // holding a claimed chunk while others run out would idle them).
        const bool early = (long long)c + 2ll * gridDim.x < (long long)nc;
        unsigned int next = 0u;
        if (tid == 0 && early) next = atomicAdd(ctr, 1u);
        const long long u0 = (long long)(((unsigned long long)g.n_units * c) / nc);
        const long long u1 = (long long)(((unsigned long long)g.n_units * (c + 1)) / nc);
        if (HIST == HIST_LDS && since_flush + chunk_max > (1ll << 31)) {
            // Per-slot LDS counters are 32-bit: flush before any could reach
            // 2^31 (uniform across the block).
            hist_flush(lds, a.nbins, a.copies_log2, a.hist_acc);
            __syncthreads();  // every thread's reads of LDS done before it is zeroed
            lds_zero(lds, a.nbins, a.copies_log2);
            since_flush = 0;
        }
        since_flush += chunk_max;

        Lane L = {INFINITY, -INFINITY, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        Wave W = {0.f, 0, 0ull, 0ull, 0ull};
        if (HIST == HIST_NONE || hist_on)
            scan_units<STATS, HIST, ACC, U>(g, u0, u1, L, W, H);
        else
            scan_units<STATS, HIST_NONE, ACC, U>(g, u0, u1, L, W, H);
        write_wave_record<STATS, ACC>(L, W, &ring[filled * nw + wid]);
        if (tid == 0) s_ids[filled] = c;
        __syncthreads();  // every part written; every thread has read s_chunk
        if (tid == 0) s_chunk = (int)(early ? next : atomicAdd(ctr, 1u));
        __syncthreads();
        // When the ring is full, every wavefront merges one of its chunks
        // (one merge time per nw chunks, not one per chunk on the critical
        // path), and a barrier frees the ring.
        if (++filled == nw) {
            write_chunk_record<STATS>(&ring[wid * nw], nw,
                                      reinterpret_cast<ChunkRec *>(a.recs) + s_ids[wid]);
            __syncthreads();
            filled = 0;
        }
    }
    // The chunks left in the ring (published by the loop's last barrier).
    if (wid < filled)
        write_chunk_record<STATS>(&ring[wid * nw], nw,
                                  reinterpret_cast<ChunkRec *>(a.recs) + s_ids[wid]);
    if (HIST == HIST_LDS) hist_flush(lds, a.nbins, a.copies_log2, a.hist_acc);

    if (!last_to_arrive(a.ticket, gridDim.x, &s_last)) return;

    const ChunkRec *recs = reinterpret_cast<const ChunkRec *>(a.recs);
    unsigned long long nv, below, above;
    if (STATS) {
        finish_stats<ACC, ChunkRec>(recs, nc, CUBE_ACCUM_FP64MERGE, g.n_total, a.out,
                                    a.want_range ? a.out_range : nullptr, a.nbins, nv, below,
                                    above);
    } else {
        const Summary<double> S = merge_two_sweep<ChunkRec>(recs, nc);
        nv = S.nv;
        below = S.below;
        above = S.above;
    }
    if (HIST != HIST_NONE)
        finish_hist(a.hist_acc, a.counts, a.nbins, hist_on, below, above, g.n_total - nv,
                    a.accumulate != 0);
    if (tid == 0) {
        *a.ticket = 0u;
        *ctr = 0u;
    }
}

size_t pass_lds_bytes(bool stats, int hist, int nbins, int copies_log2, int threads,
                      bool dynamic)
{
    (void)stats;
    if (dynamic) {
        const size_t nw = (size_t)threads / 64;
        return (size_t)dyn_ring_offset_words(hist == HIST_LDS, nbins, copies_log2) * 4u +
               nw * nw * sizeof(WaveRec);
    }
    if (hist == HIST_LDS || hist == HIST_HOT)
        return (size_t)(nbins + 2) * ((size_t)1 << copies_log2) * 4u;
    return 0;
}

template <bool STATS, int HIST, int ACC>
static const void *kernel_of(int unroll)
{
    if (unroll == 2) return reinterpret_cast<const void *>(&k_pass<STATS, HIST, ACC, 2>);
    return reinterpret_cast<const void *>(&k_pass<STATS, HIST, ACC, 4>);
}

template <bool STATS, int HIST>
static const void *dyn_kernel_of(int unroll)
{
    if (unroll == 2) return reinterpret_cast<const void *>(&k_pass_dyn<STATS, HIST, 2>);
    return reinterpret_cast<const void *>(&k_pass_dyn<STATS, HIST, 4>);
}

// The dynamic-partition kernels: FP64MERGE moments, no hot-bin form.
static const void *pick_dyn(bool stats, int hist, int u)
{
    if (stats) {
        if (hist == HIST_NONE) return dyn_kernel_of<true, HIST_NONE>(u);
        if (hist == HIST_LDS) return dyn_kernel_of<true, HIST_LDS>(u);
        return dyn_kernel_of<true, HIST_GLOBAL>(u);
    }
    if (hist == HIST_LDS) return dyn_kernel_of<false, HIST_LDS>(u);
    return dyn_kernel_of<false, HIST_GLOBAL>(u);
}

static const void *pick(bool stats, int hist, int acc, int u)
{
    const bool naive = acc == CUBE_ACCUM_NAIVE32;
    if (stats) {
        if (hist == HIST_NONE)
            return naive ? kernel_of<true, HIST_NONE, CUBE_ACCUM_NAIVE32>(u)
                         : kernel_of<true, HIST_NONE, CUBE_ACCUM_FP64MERGE>(u);
        if (hist == HIST_LDS)
            return naive ? kernel_of<true, HIST_LDS, CUBE_ACCUM_NAIVE32>(u)
                         : kernel_of<true, HIST_LDS, CUBE_ACCUM_FP64MERGE>(u);
        if (hist == HIST_HOT)
            return naive ? kernel_of<true, HIST_HOT, CUBE_ACCUM_NAIVE32>(u)
                         : kernel_of<true, HIST_HOT, CUBE_ACCUM_FP64MERGE>(u);
        return naive ? kernel_of<true, HIST_GLOBAL, CUBE_ACCUM_NAIVE32>(u)
                     : kernel_of<true, HIST_GLOBAL, CUBE_ACCUM_FP64MERGE>(u);
    }
    if (hist == HIST_LDS) return kernel_of<false, HIST_LDS, CUBE_ACCUM_FP64MERGE>(u);
    if (hist == HIST_HOT) return kernel_of<false, HIST_HOT, CUBE_ACCUM_FP64MERGE>(u);
    return kernel_of<false, HIST_GLOBAL, CUBE_ACCUM_FP64MERGE>(u);
}

int pass_blocks_per_cu(bool stats, int hist, int threads, size_t lds_bytes, int unroll,
                       bool dynamic)
{
    int n = 0;
    const void *k = dynamic && hist != HIST_HOT ? pick_dyn(stats, hist, unroll)
                                                : pick(stats, hist, CUBE_ACCUM_FP64MERGE, unroll);
    if (lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) !=
            hipSuccess)
        return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds_bytes) != hipSuccess)
        return 1;
    return n < 1 ? 1 : n;
}

hipError_t launch_pass(const PassArgs &a, bool stats, int hist, int threads, int blocks,
                       size_t lds_bytes, int unroll, hipStream_t s)
{
    if (a.n_chunks > 0 && (hist == HIST_HOT || a.accum_mode != CUBE_ACCUM_FP64MERGE))
        return hipErrorInvalidValue;  // the planner never asks for these
    const void *k = a.n_chunks > 0 ? pick_dyn(stats, hist, unroll)
                                   : pick(stats, hist, a.accum_mode, unroll);
    if (lds_bytes > 64 * 1024) {
        // More than the default dynamic LDS limit of a launch.
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    PassArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(k, dim3((unsigned)blocks), dim3((unsigned)threads), args,
                           lds_bytes, s);
}

}  // namespace cube
