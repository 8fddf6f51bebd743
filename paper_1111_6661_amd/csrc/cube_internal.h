// cube_internal.h -- structures shared by the kernels and the C-ABI layer of
// the cube statistics library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>
#include <vector>

#include "cubestats.h"

namespace cube {

// One partial result per wavefront (the local stage of the paper's two-stage
// gather, Section 2).  Moments are FP32 double-float pairs relative to the
// wavefront's pivot K; in the naive mode K = 0 and the lo parts are 0.
struct alignas(16) WaveRec {
    float K, s1h, s1l, s2h, s2l, mn, mx, pad;
    unsigned long long n_valid, below, above, pad2;
};
static_assert(sizeof(WaveRec) == 64, "WaveRec is 64 bytes");

// One partial result per chunk of a pass with a dynamic partition: the
// chunk's wavefront records merged in FP64 (count, mean, sum of squared
// deviations about the mean, extrema, below / above counts).
struct alignas(16) ChunkRec {
    double mean, m2;
    float mn, mx;
    unsigned int pad0, pad1;
    unsigned long long n_valid, below, above, pad2;
};
static_assert(sizeof(ChunkRec) == 64, "ChunkRec is 64 bytes");

// The chunk counter of a pass with a dynamic partition is this word of the
// ticket buffer (a separate 128-byte line from the ticket itself).
constexpr int CHUNK_CTR_WORD = 32;

// A histogram range as the kernels use it.  ok: 1 valid, 0 invalid range,
// 2 no valid voxel (the two-pass range of an all-blank box).
struct HistRange {
    float lo, hi, scale;
    int32_t ok;
};

// A box after merging contiguous axes: rows of `row_len` contiguous floats,
// row (y, z) starting at ptr + y*sy + z*sz.  Rows are cut into `segs`
// segments of `seg_len` floats (seg_len a multiple of 4); a unit of work is
// one segment of one row, numbered u = (z*ny + y)*segs + s.
struct Geom {
    const float *ptr;
    int64_t row_len, ny, nz, sy, sz;
    int64_t seg_len, segs, n_units;
    uint64_t n_total;
};

// Histogram modes of a pass: none; LDS sub-histograms (every in-range voxel
// one LDS atomic); 64-bit global atomics (more bins than LDS holds); and LDS
// sub-histograms with a hot bin: the block's most likely bin (the bin of the
// first in-range voxel it meets) is never written to LDS -- its count is the
// block's in-range count, known from the ballots, minus every other bin --
// so a skewed histogram costs almost no LDS atomics.
enum : int32_t { HIST_NONE = 0, HIST_LDS = 1, HIST_GLOBAL = 2, HIST_HOT = 3 };

struct PassArgs {
    Geom g;
    int32_t nbins;
    int32_t copies_log2;         // LDS sub-histogram copies = 1 << copies_log2
    HistRange range;             // the given range (when dev_range is null)
    const HistRange *dev_range;  // range formed on the device by a stats pass
    WaveRec *recs;               // gridDim.x * waves-per-block records (static
                                 // partition), or n_chunks ChunkRecs (dynamic)
    unsigned int *ticket;        // last-block-done counter and, at word
                                 // CHUNK_CTR_WORD, the chunk counter; 0 between launches
    unsigned long long *hist_acc;// nbins global accumulators, 0 between launches
    cube_stats_t *out;           // device result (stats passes)
    unsigned long long *counts;  // device counts, nbins + 3 (histogram passes)
    HistRange *out_range;        // device [min, max] range (two-pass pass 1)
    int32_t accum_mode;          // CUBE_ACCUM_*
    int32_t want_range;          // pass 1 of a two-pass call: write out_range
    int32_t accumulate;          // add the counts to `counts` instead of writing them
    int32_t n_chunks;            // 0: static partition; else chunks claimed at run time
};

// Kernel launchers (cube_kernels.hip).  `stats`: compute the statistics;
// `hist`: HIST_NONE / HIST_LDS / HIST_GLOBAL / HIST_HOT.  Returns the launch
// error.
// `unroll`: float4 loads per lane per pipelined tile (2 or 4).
hipError_t launch_pass(const PassArgs &a, bool stats, int hist, int threads,
                       int blocks, size_t lds_bytes, int unroll, hipStream_t s);

// Dynamic LDS bytes a pass needs (`dynamic`: of the dynamic-partition
// kernel, which keeps a ring of wavefront records after its histogram).
size_t pass_lds_bytes(bool stats, int hist, int nbins, int copies_log2, int threads,
                      bool dynamic = false);
// Where that ring starts in the dynamic LDS, in 32-bit words (16-byte
// aligned, after the LDS histogram if there is one).
__host__ __device__ inline int dyn_ring_offset_words(bool lds_hist, int nbins, int copies_log2)
{
    return lds_hist ? (((nbins + 2) << copies_log2) + 3) & ~3 : 0;
}

// Occupancy of one pass configuration: resident blocks per CU.
// `dynamic`: of the dynamic-partition kernel.
int pass_blocks_per_cu(bool stats, int hist, int threads, size_t lds_bytes, int unroll,
                       bool dynamic = false);

// ------------------------------------------------ host helpers (cube_capi.hip)
// A validated box: extents, pitches (defaults resolved) and voxel count.
struct Box {
    const float *ptr;
    int64_t nx, ny, nz, sy, sz;
    uint64_t n;
};

struct Plan {
    Geom g;
    int threads, blocks, copies_log2, hist, unroll;
    int chunks;  // 0: static partition; else the dynamic partition's chunk count
    size_t lds;
};

// No C++ exception leaves the C ABI: an entry point whose body may allocate
// host memory wraps it in CUBE_GUARD_BEGIN ... CUBE_GUARD_END, which turns
// std::bad_alloc into CUBE_ENOMEM and anything else into CUBE_EDEVICE.
#define CUBE_GUARD_BEGIN try {
#define CUBE_GUARD_END                                                          \
    }                                                                           \
    catch (const std::bad_alloc &)                                              \
    {                                                                           \
        return cube::fail(CUBE_ENOMEM, "host memory exhausted");                \
    }                                                                           \
    catch (...)                                                                 \
    {                                                                           \
        return cube::fail(CUBE_EDEVICE, "unexpected internal error");           \
    }

// The same for entry points that return nothing: an exception is dropped.
#define CUBE_GUARD_VOID_END                                                     \
    }                                                                           \
    catch (...)                                                                 \
    {                                                                           \
    }

// Set the calling thread's error text and return `code`.
extern thread_local std::string g_err;
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// Host-only checks of a box (no HIP call) and the checks that need HIP.
int check_box(const float *ptr, const int64_t *dims, Box *b);
int check_box_device(const Box *b);
// Validate a histogram range and form its FP32 scale.
int check_range(float lo, float hi, int32_t nbins, HistRange *r);
// Merge contiguous axes of a box into rows (segments not yet set).
void collapse(const Box &b, Geom *g);
int cu_count();
int accum_mode();
// Test knobs: the values given for `kind` in the environment variable
// CUBE_FAULT_INJECT, a comma-separated list of kind:N items in which a bare
// N repeats the kind before it ("launch:2,5,event:3,expire:1").  Read when a
// server or batch is created; they force failure paths from the host while
// every kernel still runs to its normal end.
std::vector<uint64_t> fault_inject(const char *kind);
void get_launch(int *threads, int *blocks, int *copies, int *unroll);

// The launch shape of one pass over a validated box: statistics (`stats`)
// and/or a histogram (hist_kind_req 1) of nbins bins; the explicit shape of
// cube_set_launch, else the tuned one, else the default rules.
int make_plan(const Box &b, bool stats, int hist_kind_req, int nbins, Plan *p);
// Cut the rows of a collapsed box into segments so that there are at least
// `blocks` work units (a row is never cut below 4 floats).
void cut_rows(Geom &g, long long blocks);

// One pass over a validated device box on stream `s`, with the calling
// stream's workspace: statistics (to dev_out) and/or a histogram (HIST_NONE
// or HIST_LDS requested) over `range`, or over `dev_range` when it is not
// null; with `accumulate` the counts are added to dev_counts.  The box must
// hold at least one voxel.
int run_pass(const Box &b, bool stats, bool hist, int nbins, const HistRange &range,
             const HistRange *dev_range, cube_stats_t *dev_out, unsigned long long *dev_counts,
             bool accumulate, hipStream_t s);
// Two counter words (0 between launches; a kernel that uses them returns
// them to 0) in the calling device's workspace of stream `s`, at the chunk
// counter of the single-box pass; after queueing the kernel, stream_used(s)
// records the use so that the workspace outlives it.
int stream_counter(hipStream_t s, unsigned int **ctr);
int stream_used(hipStream_t s);
// Free the calling device's workspace of stream `s` (waits for its last
// use); a library-owned stream releases it before hipStreamDestroy.
void release_ws(hipStream_t s);
// The empty-box results (n_total 0, NaN statistics, zero counts) on `s`.
int write_empty(cube_stats_t *dev_out, unsigned long long *dev_counts, int nbins, hipStream_t s);

// Release the out-of-core streaming buffers and streams (cube_host.hip).
void host_release();
// Release the projection slice partials (cube_project.hip).
void project_release();
// Release the quantile counters and tables (cube_quantile.hip).
void quant_release();

// A launch shape chosen by the autotuner (cube_tune.hip).
struct TunedShape {
    int threads, unroll, copies, blocks_per_cu;
    int hot;         // 1: the hot-bin histogram (HIST_HOT) instead of HIST_LDS
    int chunk_log2;  // 0: static partition; k: dynamic, chunks of 2^k voxels
    float ms;
};
// The calling thread's hot-bin override for later single-box histogram
// passes: -1 none (tuned or default), 0 HIST_LDS, 1 HIST_HOT.  The
// autotuner sets it per candidate.
void set_hot_override(int hot);
int hot_override();
// The calling thread's partition override for later single-box passes: -1
// none (tuned or default), 0 static, k >= 1 dynamic with chunks of 2^k
// voxels (cube_set_partition).
void set_chunk_override(int chunk_log2);
int chunk_override();
// The chunk count of a dynamic partition of n voxels into chunks of
// 2^chunk_log2 voxels (at least 1, at most the record capacity).
long long chunks_of(uint64_t n, int chunk_log2);
// The tuned shape for (pass kind CUBE_Q_*, nbins, voxels), if any.
bool tuned_shape(int kind, int nbins, uint64_t voxels, TunedShape *out);

// The batched launch's automatic rule: threads per block, float4 loads per
// lane per pipelined step, each query's tile
// size from the query's own voxel count n (2^floor_log2, doubled while it is
// below 2^cap_log2 and n needs more than 2^tiles_log2 tiles), and the LDS
// budget of the histogram copies.  One rule serves every batch, so a query's
// tiling (and with it the rounding of its moments) depends on the query
// alone, never on the batch it is in.  cube_autotune_batch tunes it.
struct BatchRule {
    int threads, unroll, floor_log2, cap_log2, tiles_log2, lds_kib;
    float ms;
};
// The default is the rule the autotuner chose on an MI355X for a mixed batch
// of 64 cubes (2 loads per step: with 4 the batched kernel spills).
constexpr BatchRule DEFAULT_BATCH_RULE = {512, 2, 17, 20, 10, 64, 0.f};
constexpr int CUBE_TUNE_BATCH = 4;  // the rule's "kind" in a saved tuning table
bool batch_rule_ok(const BatchRule &r);
// The tuned rule, if the table holds one; and the autotuner's store.
bool tuned_batch_rule(BatchRule *out);
void set_tuned_batch_rule(const BatchRule &r);
// A query's tile size (voxels) under `r`.
long long rule_tile_voxels(const BatchRule &r, unsigned long long n);

}  // namespace cube
