// cube_batch.hip -- many boxes (queries) in one persistent launch.
//
// The host cuts every query into tiles (contiguous ranges of its work units)
// and lists them: first the tiles of every query's first phase (statistics,
// fused statistics + histogram, or a histogram over a given range), then the
// second-phase tiles of the two-pass queries (the histogram over the query's
// own [min, max]).  A grid sized to the GPU's occupancy pulls tiles from one
// atomic counter until the list is exhausted.  Per tile, a block scans the
// units (the same device code as the single-box pass), writes one record per
// wavefront into the query's record range and flushes its LDS histogram into
// the query's accumulators.  The block that finishes a query's last tile of
// a phase merges that query's records in tile order (FP64) and writes its
// results; for a two-pass query it also publishes the [min, max] range, which
// releases the query's second-phase tiles.  This is the paper's batched
// service (Abstract) and its sub-cube processing (Section 3) on one GPU.
//
// Progress: a second-phase tile waits only for its own query's first phase,
// whose tiles all come earlier in the list and were therefore taken by
// running blocks that never wait; the wait is bounded anyway.  If it ever
// expires the tile is skipped, the batch's error flag and the query's own
// failure flag are raised, and the query completes marked as failed (its
// histogram is incomplete); the other queries are unaffected.  Each word of
// the range a query's first phase publishes carries the launch's epoch (a
// counter the last block of every launch advances), so a range left by an
// earlier launch -- or published after its query's second phase already
// gave up -- never releases the tiles of a later launch, graph replays
// included.  The first-phase tiles of two-pass queries, and every tile near
// the end of the list, take their ticket as soon as their writes are
// complete; every other tile takes it at the block's next tile boundary
// (nothing in the launch waits for it).
// Results of a query do not depend on the other queries of the batch (its
// tiling and merge order are its own), so a query gives the same bits alone
// and in any mix.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "cube_device.h"

namespace cube {

enum : int32_t { BQ_STATS = CUBE_Q_STATS, BQ_HIST = CUBE_Q_HIST, BQ_FUSED = CUBE_Q_FUSED,
                 BQ_MINMAX = CUBE_Q_MINMAX };

struct BatchItem {                 // read-only during a launch
    Geom g;
    int32_t kind, nbins;
    HistRange range;               // given range (HIST, FUSED)
    int32_t ntiles1, ntiles2;      // tiles of phase 1 / phase 2
    long long rec1, rec2;          // first record of each phase
    long long acc0;                // first histogram accumulator
    cube_stats_t *out;
    unsigned long long *counts;
};

struct BatchState {                // counters zero between launches
    unsigned int done1, done2;
    unsigned int failed;           // a second-phase tile gave up (this launch)
    unsigned int pad;
    // The published [min, max] range of a two-pass query: lo, hi, scale and
    // ok, each in the low half of a 64-bit word whose high half is the epoch
    // tag of the launch that published it.  A reader takes the range when
    // all four tags are its own launch's: every word is read and written
    // whole, so no fence is needed between the flag and the data.
    unsigned long long rng[4];
};

struct BatchTile {
    int32_t item, phase;
    int32_t local, pad;            // tile index within the item's phase
    long long u0, u1;              // its work units [u0, u1)
};

struct BatchArgs {
    const BatchItem *items;
    BatchState *state;
    const BatchTile *tiles;
    int32_t n_tiles, copies_log2;
    int32_t lds_words;             // the dynamic LDS histogram area
    WaveRec *recs;
    unsigned long long *acc;
    unsigned int *ctl;             // [0] next tile, [1] exit ticket, [2] error flag
                                   // (sticky until read by the host), [3] epoch
    int32_t accum_mode;
    unsigned int spin_limit;       // polls of a range wait; 0 = give up at once
    unsigned int *done_flags;      // host-mapped, one per query: `gen` once done,
                                   // with DONE_FAILED set if the query failed
    unsigned int gen;              // 1 .. 2^31 - 1
};

constexpr unsigned int DONE_FAILED = 0x80000000u;

__device__ __forceinline__ long long uniform_ll(long long v)
{
    const unsigned long long u = (unsigned long long)v;
    return (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                       (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)u));
}

template <bool STATS, int HIST, int U>
__device__ void batch_scan(const BatchItem &it, long long u0, long long u1, Lane &L, Wave &W,
                           const Hist &H)
{
    scan_units<STATS, HIST, CUBE_ACCUM_FP64MERGE, U>(it.g, u0, u1, L, W, H);
}

// The LDS histogram flush of the batched launch, which keeps its LDS
// histogram zero between tiles: each thread reads its bins' copies as
// 16-byte words (C >= 4) and writes zero back to the words it read.  Slot 0,
// where lanes outside the range add, is never read and never cleared.
// Starts with a barrier (every LDS add of the tile is done); the cleared
// words are not added to before the completion's barriers.
__device__ __forceinline__ void hist_flush_clear(unsigned int *lds, int nbins, int copies_log2,
                                                 unsigned long long *acc)
{
    __syncthreads();
    const int C = 1 << copies_log2;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        const int last = b == nbins - 1 ? 2 : 1;  // floor(u) == nbins belongs to the last bin
        unsigned int sum = 0;
        for (int k = 1; k <= last; ++k) {
            unsigned int *w = lds + ((b + k) << copies_log2);
            if (C >= 4) {
                uint4 *w4 = reinterpret_cast<uint4 *>(w);
                for (int c = 0; c < C / 4; ++c) {
                    const uint4 v = w4[c];
                    sum += (v.x + v.y) + (v.z + v.w);
                    w4[c] = make_uint4(0u, 0u, 0u, 0u);
                }
            } else {
                for (int c = 0; c < C; ++c) {
                    sum += w[c];
                    w[c] = 0u;
                }
            }
        }
        if (sum) atomicAdd(&acc[b], (unsigned long long)sum);
    }
}

// The merge of one query's phase, by the block that took its last ticket
// (after an acquire): the records in tile order (FP64), the histogram
// accumulators, and either the published range (first phase of a two-pass
// query) or the query's completion flag.  Ends with a barrier.
__device__ __forceinline__ void batch_merge(const BatchArgs &a, int item, int phase, bool hist_on,
                                         unsigned int tag, HistRange *s_out)
{
    const int tid = threadIdx.x, nw = blockDim.x >> 6;
    const BatchItem &it = a.items[item];
    BatchState *st = &a.state[item];
    const bool stats = phase == 1 && it.kind != BQ_HIST;
    const bool hist = phase == 2 || it.kind == BQ_HIST || it.kind == BQ_FUSED;
    const int ntiles = phase == 1 ? it.ntiles1 : it.ntiles2;
    const WaveRec *recs = a.recs + (phase == 1 ? it.rec1 : it.rec2);
    unsigned long long *acc = a.acc + it.acc0;
    const int n_recs = ntiles * nw;
    unsigned long long nv, below, above;
    if (stats) {
        finish_stats<CUBE_ACCUM_FP64MERGE>(recs, n_recs, a.accum_mode, it.g.n_total, it.out,
                                           it.kind == BQ_MINMAX ? s_out : nullptr, it.nbins, nv,
                                           below, above);
    } else {
        const Summary<float> S = merge_records<float, CUBE_ACCUM_KAHAN32>(recs, n_recs);
        nv = S.nv;
        below = S.below;
        above = S.above;
    }
    if (hist) finish_hist(acc, it.counts, it.nbins, hist_on, below, above, it.g.n_total - nv);
    __syncthreads();
    if (tid == 0) {
        bool finished = true;
        unsigned int failed = 0u;
        if (phase == 1) {
            st->done1 = 0u;
            if (it.kind == BQ_MINMAX) {
                // Publish the range, each word tagged with this launch.
                finished = false;
                const HistRange r = *s_out;
                const unsigned long long t = (unsigned long long)tag << 32;
                __hip_atomic_store(&st->rng[0], t | __float_as_uint(r.lo), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&st->rng[1], t | __float_as_uint(r.hi), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&st->rng[2], t | __float_as_uint(r.scale), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&st->rng[3], t | (unsigned int)r.ok, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            // Every second-phase tile of this query has arrived: its counters
            // return to zero.  The range words need no reset (the next launch
            // waits for its own tag).
            failed = st->failed;
            st->failed = 0u;
            st->done2 = 0u;
        }
        if (finished && a.done_flags) {
            // The query's outputs are complete: tell the host (a system-scope
            // release store orders the outputs first).
            __hip_atomic_store(&a.done_flags[item], a.gen | (failed ? DONE_FAILED : 0u),
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    // The merge's shared memory is reused by the next tile.
    __syncthreads();
}

// U: float4 loads per lane per pipelined tile step (2 or 4, the rule's).
template <int U>
__global__ void __launch_bounds__(1024) k_batch(BatchArgs a)
{
    extern __shared__ __align__(16) unsigned int lds[];
    __shared__ int s_tile, s_next;
    __shared__ BatchTile s_desc;
    __shared__ unsigned int s_flag, s_last, s_tag;
    __shared__ HistRange s_range, s_pub;
    const int tid = threadIdx.x, wid = tid >> 6, nw = blockDim.x >> 6;
    const long long ahead_span = 2ll * gridDim.x;

    // Tiles are claimed by thread 0 at the end of the previous tile, in the
    // same round trip as the tickets, and the claimed tile's descriptor is
    // staged in LDS there, so a tile starts without waiting on memory.  While
    // more than two grids' worth of tiles lie beyond the next tile, the block
    // also holds the tile after it (claimed one tile ahead: its claim then
    // needs no answer from the claim before it).  Nearer the end of the list
    // a block holds no tile that an idle block could be working on (a short
    // batch would otherwise run on half its blocks, two tiles each).  A
    // first-phase tile held ahead is always held by a block working on an
    // earlier first-phase tile (every first-phase tile precedes every
    // second-phase tile in the list), which never waits, so every first-phase
    // tile is still processed and second-phase waits end.
    if (tid == 0) {
        // This launch's epoch tag (never 0).  The epoch only changes when the
        // last block leaves, after every block has read it here.
        s_tag = (__hip_atomic_load(&a.ctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                 0x7fffffffu) + 1u;
        // With more than four grids' worth of tiles, every first claim
        // (below two grids) leaves more than two grids beyond the tile after
        // it: one claim of two consecutive tiles takes both.
        const bool two = (long long)a.n_tiles > 2ll * ahead_span;
        const int t0 = (int)atomicAdd(&a.ctl[0], two ? 2u : 1u);
        s_next = two ? t0 + 1 : -1;
        if (t0 < a.n_tiles) s_desc = a.tiles[t0];
        s_tile = t0;
    }
    // The LDS histogram is zero between tiles (each flush clears what it
    // read), so it is cleared once here.
    for (int i = tid; i < a.lds_words; i += blockDim.x) lds[i] = 0u;
    __syncthreads();
    const unsigned int tag = s_tag;

    // The ticket of a tile whose completion releases nothing inside the
    // launch (every tile but the first-phase tiles of two-pass queries) is
    // taken one tile late, at the next tile's end, while the block holds a
    // tile ahead (so it has a next tile): by then its writes are long
    // complete, so no wave waits for them.  Nearer the end of the list every
    // tile takes its ticket at once, so no merge waits for the block's exit.
    // Pending: its query and phase (uniform), or item -1.
    int pend_item = -1, pend_phase = 0;
    bool pend_hist_on = false;

    while (true) {
        // Uniform values (scalar registers): one address per wavefront for
        // the item's fields and the tile's bounds.
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        const bool more = t < a.n_tiles;
        const bool held = __builtin_amdgcn_readfirstlane(s_next) >= 0;
        int item = 0, phase = 1, local = 0;
        bool sync = false, hist_on = false;
        if (more) {
            item = __builtin_amdgcn_readfirstlane(s_desc.item);
            phase = __builtin_amdgcn_readfirstlane(s_desc.phase);
            local = __builtin_amdgcn_readfirstlane(s_desc.local);
            const BatchItem &it = a.items[item];
            BatchState *st = &a.state[item];
            const long long u0 = uniform_ll(s_desc.u0), u1 = uniform_ll(s_desc.u1);
            unsigned long long *acc = a.acc + it.acc0;

            // The histogram range of this tile.
            HistRange range = it.range;
            bool skip = false;
            if (phase == 2) {
                if (tid == 0) {
                    // Relaxed polls of the four tagged words.  A spin limit of
                    // 0 (a test setting) gives up at once.
                    unsigned int spins = 0;
                    unsigned long long w[4];
                    s_flag = 1u;
                    while (true) {
                        bool up = a.spin_limit != 0u;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            w[k] = __hip_atomic_load(&st->rng[k], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                            up = up && (unsigned int)(w[k] >> 32) == tag;
                        }
                        if (up) break;
                        if (a.spin_limit == 0u || ++spins > a.spin_limit) {
                            atomicOr(&a.ctl[2], 1u);
                            atomicOr(&st->failed, 1u);
                            s_flag = 0u;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                    if (s_flag) {
                        HistRange r;
                        r.lo = __uint_as_float((unsigned int)w[0]);
                        r.hi = __uint_as_float((unsigned int)w[1]);
                        r.scale = __uint_as_float((unsigned int)w[2]);
                        r.ok = (int32_t)(unsigned int)w[3];
                        s_range = r;
                    }
                }
                __syncthreads();
                skip = s_flag == 0u;
                range = s_range;
            }
            const bool stats = phase == 1 && it.kind != BQ_HIST;
            const bool hist = phase == 2 || it.kind == BQ_HIST || it.kind == BQ_FUSED;
            sync = (phase == 1 && it.kind == BQ_MINMAX) || !held;

            Hist H;
            hist_on = hist && range.ok == 1;
            hist_setup(H, range, it.nbins, a.copies_log2, lds, acc);
            Lane L = {INFINITY, -INFINITY, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            Wave W = {0.f, 0, 0ull, 0ull, 0ull};
            if (!skip) {
                if (stats && hist_on)
                    batch_scan<true, HIST_LDS, U>(it, u0, u1, L, W, H);
                else if (stats)
                    batch_scan<true, HIST_NONE, U>(it, u0, u1, L, W, H);
                else if (hist_on)
                    batch_scan<false, HIST_LDS, U>(it, u0, u1, L, W, H);
                else  // an invalid [min, max] range bins nothing
                    batch_scan<false, HIST_NONE, U>(it, u0, u1, L, W, H);
            }
            // The pending tile's writes, issued a tile ago, are complete
            // before this tile's are issued.
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            WaveRec *recs = a.recs + (phase == 1 ? it.rec1 : it.rec2);
            if (stats)
                write_wave_record<true, CUBE_ACCUM_FP64MERGE, true>(
                    L, W, &recs[(long long)local * nw + wid]);
            else
                write_wave_record<false, CUBE_ACCUM_FP64MERGE, true>(
                    L, W, &recs[(long long)local * nw + wid]);
            if (hist) hist_flush_clear(lds, it.nbins, a.copies_log2, acc);
            // A tile that takes its ticket now waits for its own writes.
            if (sync) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        } else {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        if (!more && pend_item < 0) break;

        // Completion.  The records are written through the L2 and the counts
        // are atomics: once every wavefront has waited for its own writes,
        // they are performed at device scope, and a ticket needs no L2
        // write-back (see last_to_arrive_wt).  Thread 0 sends the tickets,
        // the claim and the next descriptor's load together.
        __syncthreads();
        if (tid == 0) {
            unsigned int last = 0u;
            if (pend_item >= 0) {
                const BatchItem &ip = a.items[pend_item];
                BatchState *sp = &a.state[pend_item];
                const unsigned int tk = atomicAdd(pend_phase == 1 ? &sp->done1 : &sp->done2, 1u);
                if (tk == (unsigned int)(pend_phase == 1 ? ip.ntiles1 : ip.ntiles2) - 1u)
                    last |= 1u;
            }
            if (more) {
                if (sync) {
                    const BatchItem &it = a.items[item];
                    BatchState *st = &a.state[item];
                    const unsigned int tk = atomicAdd(phase == 1 ? &st->done1 : &st->done2, 1u);
                    if (tk == (unsigned int)(phase == 1 ? it.ntiles1 : it.ntiles2) - 1u)
                        last |= 2u;
                }
                int nxt = s_next, ahead = -1;
                if (nxt >= 0) {
                    if ((long long)nxt + ahead_span < (long long)a.n_tiles)
                        ahead = (int)atomicAdd(&a.ctl[0], 1u);
                } else {
                    nxt = (int)atomicAdd(&a.ctl[0], 1u);
                }
                if (nxt < a.n_tiles) s_desc = a.tiles[nxt];
                s_tile = nxt;
                s_next = ahead;
            }
            if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_last = last;
        }
        __syncthreads();
        const unsigned int last = s_last;
        if (last & 1u) batch_merge(a, pend_item, pend_phase, pend_hist_on, tag, &s_pub);
        if (last & 2u) batch_merge(a, item, phase, hist_on, tag, &s_pub);
        if (!more) break;
        pend_item = sync ? -1 : item;
        pend_phase = phase;
        pend_hist_on = hist_on;
    }

    // The last block to leave returns the work counters to zero and starts
    // the next epoch.
    if (tid == 0 && atomicAdd(&a.ctl[1], 1u) == gridDim.x - 1) {
        a.ctl[0] = 0u;
        a.ctl[1] = 0u;
        __hip_atomic_store(&a.ctl[3], (tag & 0x7fffffffu), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ host side
long long rule_tile_voxels(const BatchRule &r, unsigned long long n)
{
    long long tv = (long long)1 << r.floor_log2;
    while (tv < ((long long)1 << r.cap_log2) && (unsigned long long)tv << r.tiles_log2 < n)
        tv <<= 1;
    return tv;
}

static const void *batch_kernel(int unroll)
{
    return unroll == 2 ? reinterpret_cast<const void *>(&k_batch<2>)
                       : reinterpret_cast<const void *>(&k_batch<4>);
}

static hipError_t batch_occupancy(int threads, int unroll, size_t lds, int *bpc)
{
    const void *k = batch_kernel(unroll);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k, threads, lds);
}

}  // namespace cube

using namespace cube;

// The batch object: device buffers sized for the largest batch seen so far,
// pinned staging for the work list, and a captured graph per stream.
struct cube_batch {
    std::mutex mu;
    int device = 0;
    // capacities
    size_t cap_items = 0, cap_tiles = 0, cap_recs = 0, cap_acc = 0;
    BatchItem *d_items = nullptr;
    BatchState *d_state = nullptr;
    BatchTile *d_tiles = nullptr;
    WaveRec *d_recs = nullptr;
    unsigned long long *d_acc = nullptr;
    unsigned int *d_ctl = nullptr;
    BatchItem *h_items = nullptr;   // pinned
    BatchTile *h_tiles = nullptr;   // pinned
    hipStream_t last_stream = nullptr;
    hipEvent_t staged = nullptr;    // the last work-list copy has been read
    hipEvent_t launched = nullptr;  // recorded after every launch of the batch
    unsigned int *h_done = nullptr; // host-mapped per-query completion flags
    unsigned int *d_done = nullptr; // the same memory as the device sees it
    size_t cap_done = 0;
    unsigned int gen = 0;
    uint64_t launches = 0;          // launches of this batch so far
    std::vector<uint64_t> expire;   // test knob: launches whose range waits give up
    int order = 0;                  // 0 largest queries first, 1 smallest first
    bool have_work = false;
    BatchArgs args;
    int threads_req = 0;             // 0: the rule's
    int threads = 512, blocks = 0;   // of the current work list
    int unroll = 4;                  // of the current work list (the rule's)
    size_t lds = 0;
    long long tile_voxels = 1 << 20; // 0: the rule's, per query
    bool have_rule = false;          // the autotuner's candidate, else the table's
    BatchRule rule = DEFAULT_BATCH_RULE;
    hipGraph_t graph = nullptr;       // the launch, captured once per work list;
    hipGraphExec_t graph_exec = nullptr;  // replayed on any stream
};

namespace {

void drop_graph(cube_batch *b)
{
    if (!b->graph_exec && !b->graph) return;
    // A replay may still be running: the last launch's event covers it
    // (launches of a batch are ordered).
    if (b->launched) hipEventSynchronize(b->launched);
    if (b->graph_exec) hipGraphExecDestroy(b->graph_exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

void free_buffers(cube_batch *b)
{
    if (b->last_stream || b->have_work) hipStreamSynchronize(b->last_stream);
    hipFree(b->d_items);
    hipFree(b->d_state);
    hipFree(b->d_tiles);
    hipFree(b->d_recs);
    hipFree(b->d_acc);
    hipFree(b->d_ctl);
    hipHostFree(b->h_items);
    hipHostFree(b->h_tiles);
    b->d_items = nullptr;
    b->d_state = nullptr;
    b->d_tiles = nullptr;
    b->d_recs = nullptr;
    b->d_acc = nullptr;
    b->d_ctl = nullptr;
    b->h_items = nullptr;
    b->h_tiles = nullptr;
    b->cap_items = b->cap_tiles = b->cap_recs = b->cap_acc = 0;
}

// Grow the buffers to hold the given sizes (waits for the previous launch;
// new state / accumulators / counters are zeroed).
int ensure(cube_batch *b, size_t items, size_t tiles, size_t recs, size_t acc)
{
    if (items <= b->cap_items && tiles <= b->cap_tiles && recs <= b->cap_recs &&
        acc <= b->cap_acc)
        return CUBE_OK;
    drop_graph(b);
    free_buffers(b);
    items = items < 64 ? 64 : items * 3 / 2;
    tiles = tiles < 1024 ? 1024 : tiles * 3 / 2;
    recs = recs < 4096 ? 4096 : recs * 3 / 2;
    acc = acc < 4096 ? 4096 : acc * 3 / 2;
    bool ok = hipMalloc(&b->d_items, items * sizeof(BatchItem)) == hipSuccess &&
              hipMalloc(&b->d_state, items * sizeof(BatchState)) == hipSuccess &&
              hipMalloc(&b->d_tiles, tiles * sizeof(BatchTile)) == hipSuccess &&
              hipMalloc(&b->d_recs, recs * sizeof(WaveRec)) == hipSuccess &&
              hipMalloc(&b->d_acc, acc * 8) == hipSuccess &&
              hipMalloc(&b->d_ctl, 256) == hipSuccess &&
              hipHostMalloc(&b->h_items, items * sizeof(BatchItem)) == hipSuccess &&
              hipHostMalloc(&b->h_tiles, tiles * sizeof(BatchTile)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_buffers(b);
        return fail(CUBE_ENOMEM, "batch buffer allocation failed");
    }
    hipError_t e;
    if ((e = hipMemset(b->d_state, 0, items * sizeof(BatchState))) != hipSuccess ||
        (e = hipMemset(b->d_acc, 0, acc * 8)) != hipSuccess ||
        (e = hipMemset(b->d_ctl, 0, 256)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
        free_buffers(b);
        return hip_fail(e, "batch buffer initialisation");
    }
    b->cap_items = items;
    b->cap_tiles = tiles;
    b->cap_recs = recs;
    b->cap_acc = acc;
    return CUBE_OK;
}

// Host-mapped completion flags for `n` queries (kept, grown on demand).
int ensure_done(cube_batch *b, size_t n)
{
    if (n <= b->cap_done) return CUBE_OK;
    if (b->have_work) hipStreamSynchronize(b->last_stream);
    if (b->h_done) hipHostFree(b->h_done);
    b->h_done = nullptr;
    b->d_done = nullptr;
    b->cap_done = 0;
    const size_t cap = n < 256 ? 256 : n * 2;
    hipError_t e;
    if ((e = hipHostMalloc(&b->h_done, cap * 4, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
        return hip_fail(e, "completion flags");
    memset(b->h_done, 0, cap * 4);
    if ((e = hipHostGetDevicePointer((void **)&b->d_done, b->h_done, 0)) != hipSuccess)
        return hip_fail(e, "completion flags (device view)");
    b->cap_done = cap;
    return CUBE_OK;
}

// Launches of one batch share its device state: a launch on another stream
// than the previous one waits (on the device) for that one to finish.
hipError_t order_after_previous(cube_batch *b, hipStream_t s)
{
    if (!b->launched) return hipSuccess;
    return b->last_stream == s ? hipSuccess : hipStreamWaitEvent(s, b->launched, 0);
}

hipError_t mark_launched(cube_batch *b, hipStream_t s)
{
    hipError_t e;
    if (!b->launched &&
        (e = hipEventCreateWithFlags(&b->launched, hipEventDisableTiming)) != hipSuccess)
        return e;
    b->last_stream = s;
    return hipEventRecord(b->launched, s);
}

int launch_batch(cube_batch *b, hipStream_t s)
{
    // A new generation per launch (31 bits; the top bit of a flag marks a
    // failed query): completion flags of earlier launches never read as done.
    b->gen = (b->gen + 1u) & 0x7fffffffu;
    if (b->gen == 0) b->gen = 1u;
    b->args.gen = b->gen;
    BatchArgs a = b->args;
    ++b->launches;
    for (uint64_t n : b->expire)
        if (n == b->launches) a.spin_limit = 0u;
    void *args[] = {&a};
    hipError_t e = order_after_previous(b, s);
    if (e != hipSuccess) return hip_fail(e, "batch ordering");
    e = hipLaunchKernel(batch_kernel(b->unroll), dim3(b->blocks), dim3(b->threads), args,
                        b->lds, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    if ((e = mark_launched(b, s)) != hipSuccess) return hip_fail(e, "batch event");
    return CUBE_OK;
}

}  // namespace

extern "C" {

int cube_batch_create(cube_batch_t **out)
{
    CUBE_GUARD_BEGIN
    if (!out) return fail(CUBE_EINVAL, "out is NULL");
    cube_batch *b = new cube_batch;
    hipGetDevice(&b->device);
    // Test knob: CUBE_FAULT_INJECT="expire:N[,M...]": in launches N, M, ...
    // of this batch (counted from 1; enqueues and relaunches) every range
    // wait gives up at once, so every two-pass query of them fails.
    b->expire = fault_inject("expire");
    *out = b;
    return CUBE_OK;
    CUBE_GUARD_END
}

void cube_batch_destroy(cube_batch_t *b)
{
    CUBE_GUARD_BEGIN
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        drop_graph(b);
        free_buffers(b);
        if (b->staged) hipEventDestroy(b->staged);
        if (b->launched) hipEventDestroy(b->launched);
        if (b->h_done) hipHostFree(b->h_done);
    }
    delete b;
    CUBE_GUARD_VOID_END
}

int cube_batch_set_tile(cube_batch_t *b, int64_t tile_voxels, int32_t threads)
{
    if (!b) return fail(CUBE_EINVAL, "batch is NULL");
    if (tile_voxels != 0 && (tile_voxels < 4096 || tile_voxels > ((int64_t)1 << 30)))
        return fail(CUBE_EINVAL, "tile_voxels outside [4096, 2^30] (or 0 for automatic)");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(CUBE_EINVAL, "threads must be 0, 256, 512 or 1024");
    std::lock_guard<std::mutex> lk(b->mu);
    b->tile_voxels = tile_voxels;
    b->threads_req = threads;
    return CUBE_OK;
}

int cube_batch_enqueue(cube_batch_t *b, const cube_query_t *q, int32_t n, void *stream)
{
    CUBE_GUARD_BEGIN
    if (!b) return fail(CUBE_EINVAL, "batch is NULL");
    if (n < 0 || (n > 0 && !q)) return fail(CUBE_EINVAL, "bad query list");
    std::lock_guard<std::mutex> lk(b->mu);
    hipStream_t s = (hipStream_t)stream;
    // Validate every query and plan its tiles.
    std::vector<BatchItem> items((size_t)n);
    std::vector<long long> order((size_t)n);
    std::vector<long long> upts((size_t)n);  // work units per tile
    size_t n_tiles = 0, n_recs = 0, n_acc = 0;
    int max_bins = 1;
    // The automatic rule: the autotuner's candidate, else the tuned one,
    // else the defaults.
    BatchRule rule = DEFAULT_BATCH_RULE;
    if (b->have_rule)
        rule = b->rule;
    else
        tuned_batch_rule(&rule);
    b->threads = b->threads_req ? b->threads_req : rule.threads;
    b->unroll = rule.unroll;
    const int nw = b->threads / 64;
    for (int i = 0; i < n; ++i) {
        const cube_query_t &qq = q[i];
        Box box;
        int rc = check_box(qq.ptr, qq.dims, &box);
        if (!rc) rc = check_box_device(&box);
        if (rc) return fail(rc, "query %d: %s", i, cube_last_error());
        BatchItem &it = items[(size_t)i];
        memset(&it, 0, sizeof it);
        it.kind = qq.kind;
        it.nbins = qq.nbins;
        if (qq.kind < CUBE_Q_STATS || qq.kind > CUBE_Q_MINMAX)
            return fail(CUBE_EINVAL, "query %d: unknown kind %d", i, qq.kind);
        const bool has_stats = qq.kind != CUBE_Q_HIST;
        const bool has_hist = qq.kind != CUBE_Q_STATS;
        if (has_hist) {
            if (qq.nbins < 1 || qq.nbins > 32768)
                return fail(CUBE_EINVAL, "query %d: batched histograms take 1..32768 bins", i);
            if (qq.kind == CUBE_Q_HIST || qq.kind == CUBE_Q_FUSED) {
                if ((rc = check_range(qq.lo, qq.hi, qq.nbins, &it.range)))
                    return fail(rc, "query %d: %s", i, cube_last_error());
            }
            if (!qq.counts) return fail(CUBE_EINVAL, "query %d: counts is NULL", i);
            if (qq.nbins > max_bins) max_bins = qq.nbins;
        } else {
            it.nbins = 1;
        }
        if (has_stats && !qq.out) return fail(CUBE_EINVAL, "query %d: out is NULL", i);
        it.out = qq.out;
        it.counts = (unsigned long long *)qq.counts;
        collapse(box, &it.g);
        // The query's tile size: the batch's, or (0) one from the query's own
        // size by the rule (by default at most 1024 tiles of 2^17 to 2^20
        // voxels: smaller tiles pay the per-tile completion, the record
        // stores and a ticket, more often than the parallelism repays).  Either way a
        // query's tiling depends only on itself, so its results are the same
        // alone and in any mix.
        long long tv = b->tile_voxels;
        if (tv == 0) tv = rule_tile_voxels(rule, box.n);
        // Segments of at most one tile; whole rows per tile when rows are short.
        Geom &g = it.g;
        long long seg = g.row_len < tv ? g.row_len : tv;
        seg = (seg + 3) & ~3LL;
        if (seg < 4) seg = 4;
        g.seg_len = seg;
        g.segs = box.n == 0 ? 1 : (g.row_len + seg - 1) / seg;
        g.n_units = box.n == 0 ? 0 : g.ny * g.nz * g.segs;
        long long upt = tv / seg;
        if (upt < 1) upt = 1;
        upts[(size_t)i] = upt;
        const long long nt = g.n_units == 0 ? 1 : (g.n_units + upt - 1) / upt;
        if (nt > 0x7fffffffLL) return fail(CUBE_EINVAL, "query %d: too many tiles", i);
        it.ntiles1 = (int32_t)nt;
        it.ntiles2 = qq.kind == CUBE_Q_MINMAX ? (int32_t)nt : 0;
        it.rec1 = (long long)n_recs;
        n_recs += (size_t)nt * nw;
        it.rec2 = (long long)n_recs;
        n_recs += (size_t)it.ntiles2 * nw;
        it.acc0 = (long long)n_acc;
        n_acc += has_hist ? (size_t)qq.nbins : 0;
        n_tiles += (size_t)(it.ntiles1 + it.ntiles2);
        order[(size_t)i] = i;
    }
    // Launch shape: one histogram copy layout for the batch, a grid of
    // resident blocks.
    hipError_t e;
    int clog = 0;
    const size_t lds_budget = (size_t)rule.lds_kib * 1024;
    while (clog < 5 && ((size_t)(max_bins + 2) << (clog + 1)) * 4 <= lds_budget) ++clog;
    b->lds = ((size_t)(max_bins + 2) << clog) * 4;
    int bpc = 1;
    if ((e = batch_occupancy(b->threads, b->unroll, b->lds, &bpc)) != hipSuccess)
        return hip_fail(e, "batch occupancy");
    if (bpc < 1) bpc = 1;
    const long long grid = (long long)cu_count() * bpc;
    // Work list: phase-1 tiles, largest queries first, then phase-2 tiles in
    // the same order.
    std::vector<long long> sz((size_t)n);
    for (int i = 0; i < n; ++i) sz[(size_t)i] = items[(size_t)i].ntiles1;
    if (b->order == 0)
        std::stable_sort(order.begin(), order.end(),
                         [&](long long x, long long y) { return sz[(size_t)x] > sz[(size_t)y]; });
    else
        std::stable_sort(order.begin(), order.end(),
                         [&](long long x, long long y) { return sz[(size_t)x] < sz[(size_t)y]; });
    if (n_tiles > (size_t)0x7fffffff) return fail(CUBE_EINVAL, "too many tiles");
    int rc = ensure(b, (size_t)n, n_tiles, n_recs, n_acc);
    if (rc) return rc;
    drop_graph(b);
    if ((rc = ensure_done(b, (size_t)n))) return rc;
    // A launch still running on another stream reads the device work list:
    // wait for it.  On the same stream, stream order protects the device
    // buffers; the pinned staging must still have been read by the previous
    // copy before it is rewritten.
    if (b->have_work && b->last_stream != s) hipStreamSynchronize(b->last_stream);
    if (b->staged) hipEventSynchronize(b->staged);
    size_t k = 0;
    for (int phase = 1; phase <= 2; ++phase)
        for (long long i : order) {
            const BatchItem &it = items[(size_t)i];
            const long long upt = upts[(size_t)i];
            const int nt = phase == 1 ? it.ntiles1 : it.ntiles2;
            for (int t = 0; t < nt; ++t) {
                BatchTile &bt = b->h_tiles[k++];
                bt.item = (int32_t)i;
                bt.phase = phase;
                bt.local = t;
                bt.pad = 0;
                bt.u0 = (long long)t * upt;
                bt.u1 = std::min<long long>(bt.u0 + upt, it.g.n_units);
            }
        }
    memcpy(b->h_items, items.data(), (size_t)n * sizeof(BatchItem));
    if (n > 0 &&
        ((e = hipMemcpyAsync(b->d_items, b->h_items, (size_t)n * sizeof(BatchItem),
                             hipMemcpyHostToDevice, s)) != hipSuccess ||
         (e = hipMemcpyAsync(b->d_tiles, b->h_tiles, n_tiles * sizeof(BatchTile),
                             hipMemcpyHostToDevice, s)) != hipSuccess))
        return hip_fail(e, "work-list copy");
    if (n > 0) {
        if (!b->staged && (e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "event");
        if ((e = hipEventRecord(b->staged, s)) != hipSuccess) return hip_fail(e, "event record");
    }
    long long blocks = grid;
    if (blocks > (long long)n_tiles) blocks = (long long)n_tiles;
    if (blocks < 1) blocks = 1;
    b->blocks = (int)blocks;
    BatchArgs &a = b->args;
    a.items = b->d_items;
    a.state = b->d_state;
    a.tiles = b->d_tiles;
    a.n_tiles = (int32_t)n_tiles;
    a.copies_log2 = clog;
    a.lds_words = (int32_t)(b->lds / 4);
    a.recs = b->d_recs;
    a.acc = b->d_acc;
    a.ctl = b->d_ctl;
    a.accum_mode = CUBE_ACCUM_FP64MERGE;
    a.spin_limit = 1u << 24;
    a.done_flags = b->d_done;
    b->have_work = n > 0;
    if (!b->have_work) return CUBE_OK;
    return launch_batch(b, s);
    CUBE_GUARD_END
}

int cube_batch_set_order(cube_batch_t *b, int32_t order)
{
    if (!b) return fail(CUBE_EINVAL, "batch is NULL");
    if (order != CUBE_ORDER_LARGEST_FIRST && order != CUBE_ORDER_SMALLEST_FIRST)
        return fail(CUBE_EINVAL, "unknown order %d", order);
    std::lock_guard<std::mutex> lk(b->mu);
    b->order = order == CUBE_ORDER_SMALLEST_FIRST ? 1 : 0;
    return CUBE_OK;
}

int cube_batch_query_done(cube_batch_t *b, int32_t i)
{
    if (!b || i < 0 || (size_t)i >= b->cap_done || !b->h_done) return 0;
    const unsigned int v = __atomic_load_n(&b->h_done[i], __ATOMIC_ACQUIRE);
    if ((v & ~DONE_FAILED) != b->args.gen) return 0;
    if (v & DONE_FAILED)
        return fail(CUBE_EDEVICE, "query %d: its bounded wait for its [min, max] range "
                                  "expired; its histogram is incomplete", i);
    return 1;
}

int cube_batch_relaunch(cube_batch_t *b, void *stream)
{
    CUBE_GUARD_BEGIN
    if (!b) return fail(CUBE_EINVAL, "batch is NULL");
    std::lock_guard<std::mutex> lk(b->mu);
    if (!b->have_work) return CUBE_OK;
    return launch_batch(b, (hipStream_t)stream);
    CUBE_GUARD_END
}

int cube_batch_graph_launch(cube_batch_t *b, void *stream)
{
    CUBE_GUARD_BEGIN
    if (!b) return fail(CUBE_EINVAL, "batch is NULL");
    std::lock_guard<std::mutex> lk(b->mu);
    if (!b->have_work) return CUBE_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!b->graph_exec) {
        // Capture on a private stream (a legacy default stream cannot be
        // captured), then replay the graph on the caller's stream.
        hipStream_t cap;
        if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "capture stream");
        if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            hipStreamDestroy(cap);
            return hip_fail(e, "begin capture");
        }
        BatchArgs a = b->args;
        void *args[] = {&a};
        e = hipLaunchKernel(batch_kernel(b->unroll), dim3(b->blocks), dim3(b->threads), args,
                            b->lds, cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &g);
        hipStreamDestroy(cap);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_fail(e != hipSuccess ? e : e2, "graph capture");
        }
        hipGraphExec_t ge = nullptr;
        if ((e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) != hipSuccess) {
            hipGraphDestroy(g);
            return hip_fail(e, "graph instantiate");
        }
        b->graph = g;
        b->graph_exec = ge;
    }
    if ((e = order_after_previous(b, s)) != hipSuccess) return hip_fail(e, "batch ordering");
    if ((e = hipGraphLaunch(b->graph_exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
    if ((e = mark_launched(b, s)) != hipSuccess) return hip_fail(e, "batch event");
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_batch_check(cube_batch_t *b)
{
    if (!b) return fail(CUBE_EINVAL, "batch is NULL");
    std::lock_guard<std::mutex> lk(b->mu);
    if (!b->d_ctl) return CUBE_OK;
    unsigned int ctl[4] = {0, 0, 0, 0};
    hipError_t e;
    if (b->have_work && (e = hipStreamSynchronize(b->last_stream)) != hipSuccess)
        return hip_fail(e, "batch synchronize");
    if ((e = hipMemcpy(ctl, b->d_ctl, sizeof ctl, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "batch status copy");
    if (ctl[2]) {
        // Reported once: the flag is cleared for the launches that follow.
        const unsigned int zero = 0u;
        if ((e = hipMemcpy(b->d_ctl + 2, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "batch status reset");
        return fail(CUBE_EDEVICE, "a batched two-pass query timed out waiting for its "
                                  "range; its histogram is incomplete");
    }
    return CUBE_OK;
}

int cube_autotune_batch(const cube_query_t *q, int32_t n, int32_t reps, char *report,
                        size_t report_cap)
{
    CUBE_GUARD_BEGIN
    if (n < 1 || !q) return fail(CUBE_EINVAL, "autotune needs at least one query");
    if (reps < 1 || reps > 100) return fail(CUBE_EINVAL, "reps outside [1, 100]");
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "tune stream");
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        hipStreamDestroy(s);
        return hip_fail(e, "tune events");
    }
    cube_batch_t *b = nullptr;
    int rc = cube_batch_create(&b);
    // Block sizes 256 and 512 only: a 1024-thread block fills all of a CU's
    // wavefront slots, so the concurrent batches of a server (one per slot
    // stream) could no longer share CUs -- it won a lone batch by 10 % and
    // lost the served p50 by 70 % (5.3 -> 9.0 ms on the serving mix).
    std::vector<BatchRule> cands;
    for (int th : {256, 512})
        for (int un : {2, 4})
            for (int fl : {16, 17, 18})
                for (int cp : {19, 20, 21})
                    for (int tl : {8, 9, 10})
                        for (int kib : {64, 128})
                            cands.push_back(BatchRule{th, un, fl, cp, tl, kib, 0.f});
    BatchRule best = DEFAULT_BATCH_RULE, worst = DEFAULT_BATCH_RULE;
    best.ms = 1e30f;
    worst.ms = -1.f;
    for (size_t i = 0; !rc && i < cands.size(); ++i) {
        BatchRule &c = cands[i];
        {
            std::lock_guard<std::mutex> lk(b->mu);
            b->have_rule = true;
            b->rule = c;
            b->tile_voxels = 0;
            b->threads_req = 0;
        }
        // enqueue launches once (warm-up); the first graph launch captures
        if ((rc = cube_batch_enqueue(b, q, n, s))) break;
        if ((rc = cube_batch_graph_launch(b, s))) break;
        if ((e = hipEventRecord(e0, s)) != hipSuccess) { rc = hip_fail(e, "tune event"); break; }
        for (int k = 0; k < reps && !rc; ++k) rc = cube_batch_graph_launch(b, s);
        if (rc) break;
        if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
            rc = hip_fail(e, "tune synchronize");
            break;
        }
        if ((rc = cube_batch_check(b))) break;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        c.ms = ms / reps;
        if (c.ms < best.ms) best = c;
        if (c.ms > worst.ms) worst = c;
    }
    if (b) cube_batch_destroy(b);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamDestroy(s);
    if (rc) return rc;
    set_tuned_batch_rule(best);
    if (report && report_cap) {
        char buf[512];
        auto fmt = [](const BatchRule &r, char *out, size_t cap) {
            snprintf(out, cap,
                     "{\"threads\": %d, \"unroll\": %d, \"floor_log2\": %d, \"cap_log2\": %d, "
                     "\"tiles_log2\": %d, \"lds_kib\": %d, \"ms\": %.5f}",
                     r.threads, r.unroll, r.floor_log2, r.cap_log2, r.tiles_log2, r.lds_kib,
                     r.ms);
        };
        char sb[200], sw[200];
        fmt(best, sb, sizeof sb);
        fmt(worst, sw, sizeof sw);
        snprintf(buf, sizeof buf, "{\"best\": %s, \"worst\": %s, \"candidates\": %zu}", sb, sw,
                 cands.size());
        snprintf(report, report_cap, "%s", buf);
    }
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_batch_run(const cube_query_t *q, int32_t n)
{
    CUBE_GUARD_BEGIN
    cube_batch_t *b = nullptr;
    int rc = cube_batch_create(&b);
    if (rc) return rc;
    rc = cube_batch_enqueue(b, q, n, nullptr);
    if (!rc) rc = cube_batch_check(b);
    cube_batch_destroy(b);
    return rc;
    CUBE_GUARD_END
}

}  // extern "C"
