/*
 * cubestats.h -- C ABI of the MI355X cube statistics + histogram library.
 *
 * The library computes, in one streaming pass over a float32 spectral cube
 * resident in GPU memory, the data-analysis tasks that Hassan, Fluke & Barnes
 * name for their distributed analysis service: data minimum and maximum and a
 * histogram (Abstract), and the standard deviation (Section 3, which calls it
 * a multi-pass task; here it is one pass of mergeable moments).  The paper's
 * two-stage gather (Section 2: a local stage inside a node, then a global
 * stage between nodes) becomes a local merge of per-wavefront partial results
 * followed by one global FP64 merge inside the same kernel launch.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Data: `ptr` is a DEVICE pointer (memory of the current HIP device) to
 *   float32 voxels, 4-byte aligned.  Voxel (x, y, z) of a box lives at
 *   ptr[x + sy*y + sz*z]: x fastest, the channel axis z slowest.  A dense cube
 *   has sy = nx, sz = nx*ny.  The caller owns the data; the library only reads
 *   it and never frees caller memory.
 * dims: a HOST array of 5 int64: {nx, ny, nz, sy, sz}.  sy == 0 means nx and
 *   sz == 0 means sy*ny (dense).  Rows must not overlap (sy >= nx when ny > 1)
 *   and planes must not overlap (sz >= sy*(ny-1)+nx when nz > 1).  A box with
 *   any extent 0 is legal and empty.
 * Blank voxels: any NaN bit pattern (quiet or signalling) is blank.  +-Inf are
 *   ordinary values.
 * Statistics (population): n_valid = non-blank voxels, min/max ordered with
 *   -0 < +0, mean = sum x / n_valid, m2 = sum (x-mean)^2, std = sqrt(m2/n_valid).
 *   With n_valid == 0, min/max/mean/m2/std are NaN and CUBE_NO_VALID is set.
 * Histogram over the closed range [lo, hi] with nbins bins, decided in FP32:
 *   blank -> NaN counter; x < lo -> below; x > hi -> above; otherwise bin
 *   min(nbins-1, floor((x - lo) * scale)) with scale = (float)nbins/(hi - lo),
 *   each operation one IEEE round-to-nearest FP32 operation in that order, no
 *   fused multiply-add, denormals kept.  If hi == lo every in-range voxel is
 *   bin 0.  `counts` has nbins + 3 uint64 entries: the bins, then below, above
 *   and NaN.  Counts are exact (integer atomics, order-free).
 * Valid range: lo, hi finite, hi >= lo, hi - lo finite in FP32, nbins/(hi-lo)
 *   finite in FP32 (when hi > lo), 1 <= nbins <= CUBE_MAX_BINS.
 * Precision: per-lane FP32 partial moments with compensated (TwoSum) chunk
 *   accumulation relative to a per-wavefront pivot, and one FP64 merge of the
 *   partials; mean and std agree with an FP64 evaluation of the definition to
 *   about 1e-7 relative.  Results are deterministic for a given input, shape
 *   and launch plan.
 * Errors: every int-returning entry point returns CUBE_OK (0) or a negative
 *   CUBE_E* code and never throws; cube_last_error() describes the last
 *   failure of the calling thread.  Argument errors are detected on the host
 *   before any device work is queued.
 * Streams: synchronous entry points queue on the legacy default stream (so
 *   they are ordered after work on blocking streams) and return after the
 *   result is in host memory.  *_async entry points take a hipStream_t as
 *   `void *stream` (NULL = default stream), write their results to DEVICE
 *   memory the caller owns, and return once the work is queued; the results
 *   are valid after the stream reaches that point.  Calls on different
 *   streams may run concurrently: each stream gets its own workspace.
 * Threads: all entry points are thread-safe.
 */
#ifndef CUBESTATS_H
#define CUBESTATS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every entry point below is exported; the library hides everything else. */
#if defined(__GNUC__)
#define CUBE_API __attribute__((visibility("default")))
#else
#define CUBE_API
#endif

#define CUBE_ABI_VERSION 1

#define CUBE_OK 0
#define CUBE_EINVAL (-1)  /* invalid argument (shape, pointer, range, nbins) */
#define CUBE_ENOMEM (-2)  /* a device or pinned allocation failed            */
#define CUBE_EDEVICE (-3) /* a HIP call failed; cube_last_error() names it   */
#define CUBE_EBUSY (-4)   /* a resource limit was reached (try again later)  */

#define CUBE_MAX_BINS 65536

/* cube_stats_t.flags */
#define CUBE_NO_VALID 1u        /* n_valid == 0                                */
#define CUBE_HIST_BAD_RANGE 2u  /* the [min, max] range of a two-pass call is
                                   not a valid histogram range (an infinite
                                   min or max, or a width too narrow for nbins
                                   bins); the bins are then left at zero      */

/* Accumulation modes for the moments (cube_set_accum_mode, cube_query_t). */
#define CUBE_ACCUM_FP64MERGE 0 /* default: compensated FP32 partials, FP64 merge */
#define CUBE_ACCUM_KAHAN32 1   /* same partials, final merge in FP32            */
#define CUBE_ACCUM_NAIVE32 2   /* plain FP32 sum x and sum x^2, FP32 merge      */

typedef struct cube_stats_t {
    uint64_t n_total; /* nx * ny * nz                              */
    uint64_t n_valid; /* non-blank voxels                          */
    uint64_t n_nan;   /* blank voxels                              */
    float min, max;   /* extrema of valid voxels (-0 < +0)         */
    double mean;      /* sum x / n_valid                           */
    double m2;        /* sum (x - mean)^2 (sample variance = m2/(n_valid-1)) */
    double std;       /* sqrt(m2 / n_valid), population            */
    uint32_t flags;   /* CUBE_NO_VALID | CUBE_HIST_BAD_RANGE        */
    uint32_t reserved;
} cube_stats_t; /* 64 bytes */

/* Library version; equals CUBE_ABI_VERSION of the header it was built with. */
CUBE_API int cube_abi_version(void);

/* Text of the calling thread's last error ("" if none).  Valid until the next
 * call from the same thread. */
CUBE_API const char *cube_last_error(void);

/*
 * Statistics of one box in one pass (Abstract: data minimum/maximum;
 * Section 3: standard deviation).  `stride` is NULL (dense) or a HOST array
 * {sy, sz} of pitches in elements.  `out` is HOST memory.  Synchronous.
 */
CUBE_API int cube_stats(const float *ptr, int64_t nx, int64_t ny, int64_t nz,
               const int64_t *stride, cube_stats_t *out);

/*
 * Histogram of one box over a given range (Abstract: the histogram task).
 * `counts` is HOST memory of nbins + 3 uint64.  Synchronous.
 */
CUBE_API int cube_hist(const float *ptr, const int64_t *dims, float lo, float hi,
              int32_t nbins, uint64_t *counts);

/*
 * Statistics and the histogram over a given range in ONE launch reading each
 * voxel once.  Results equal those of cube_stats and cube_hist (counts and
 * extrema bit-exact; moments within rounding).  HOST outputs.  Synchronous.
 */
CUBE_API int cube_stats_hist(const float *ptr, const int64_t *dims, float lo, float hi,
                    int32_t nbins, cube_stats_t *out, uint64_t *counts);

/*
 * Two passes: statistics, then the histogram over the data's own range
 * [min, max] (the range and its FP32 scale are formed on the device, so the
 * host never waits between the passes).  With no valid voxel the bins are 0
 * and the NaN counter holds n_total; with an invalid [min, max] range (see
 * CUBE_HIST_BAD_RANGE) the statistics are returned, the bins are 0, and the
 * call returns CUBE_EINVAL.  HOST outputs.  Synchronous.
 */
CUBE_API int cube_stats_hist_minmax(const float *ptr, const int64_t *dims, int32_t nbins,
                           cube_stats_t *out, uint64_t *counts);

/* Stream-ordered forms of the four calls above.  `dev_out` (one
 * cube_stats_t) and `dev_counts` (nbins + 3 uint64) are DEVICE memory. */
CUBE_API int cube_stats_async(const float *ptr, const int64_t *dims, cube_stats_t *dev_out,
                     void *stream);
CUBE_API int cube_hist_async(const float *ptr, const int64_t *dims, float lo, float hi,
                    int32_t nbins, uint64_t *dev_counts, void *stream);
CUBE_API int cube_stats_hist_async(const float *ptr, const int64_t *dims, float lo,
                          float hi, int32_t nbins, cube_stats_t *dev_out,
                          uint64_t *dev_counts, void *stream);
CUBE_API int cube_stats_hist_minmax_async(const float *ptr, const int64_t *dims,
                                 int32_t nbins, cube_stats_t *dev_out,
                                 uint64_t *dev_counts, void *stream);

/*
 * Allocation-free form of cube_stats_hist_async, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops
 * and harnesses that forbid hipMalloc.  Same arguments, results and errors
 * as cube_stats_hist_async (DEVICE outputs, stream-ordered on `stream`,
 * NULL = the default stream), with the same kernel; it makes no device or
 * host allocation.  Its scratch (wave records, the ticket, the histogram
 * accumulators: about 1.5 MiB) is one static device array per device, held
 * from the first call until the process ends and cleared by a small fill
 * kernel at every call.  Calls that overlap on one device (different
 * streams, or threads without ordering) race on that array and must not be
 * made.  The launch grid is narrowed to CUBE_NOALLOC_MAX_RECORDS wave
 * records (1024 blocks of 1024 threads); an explicit cube_set_launch shape
 * needing more is rejected with CUBE_EINVAL.  Under a dynamic partition
 * (cube_set_partition) the records are one per chunk: a plan with more
 * chunks is cut into CUBE_NOALLOC_MAX_RECORDS larger ones.
 */
#define CUBE_NOALLOC_MAX_RECORDS 16384
CUBE_API int cube_stats_hist_noalloc(const float *ptr, const int64_t *dims, float lo, float hi,
                                     int32_t nbins, cube_stats_t *dev_out,
                                     uint64_t *dev_counts, void *stream);

/*
 * Precision mode of the moments for later single-box calls from the CALLING
 * THREAD only (each thread starts with CUBE_ACCUM_FP64MERGE; other threads,
 * batches and the server are unaffected: batched and served queries always
 * use CUBE_ACCUM_FP64MERGE).  The FP32-only modes exist to compare against;
 * only CUBE_ACCUM_FP64MERGE meets the 1e-6 relative bound on hard inputs.
 * Returns the previous mode of the thread, or CUBE_EINVAL for an unknown
 * mode.
 */
CUBE_API int cube_set_accum_mode(int32_t mode);

/*
 * Launch-shape override for the single-box calls, used by the autotuner and
 * for experiments: threads per block (256, 512 or 1024; 0 = automatic),
 * blocks per launch (0 = automatic), histogram sub-copies per block (1..32,
 * a power of two; 0 = automatic), float4 loads per lane per pipelined tile
 * (2 or 4; 0 = automatic).  Applies to later single-box calls from the
 * CALLING THREAD only (each thread starts with all zeros).
 * Results do not depend on the launch shape except for the rounding of the
 * moments (the merge order follows the grid, or under a dynamic partition
 * the chunks).
 */
CUBE_API int cube_set_launch(int32_t threads, int32_t blocks, int32_t hist_copies, int32_t unroll);

/*
 * Form of the LDS histogram for later single-box histogram passes from the
 * CALLING THREAD (each thread starts with CUBE_HIST_AUTO):
 *   CUBE_HIST_AUTO  the autotuner's choice for the call's class, else plain;
 *   CUBE_HIST_PLAIN every in-range voxel is one LDS atomic;
 *   CUBE_HIST_HOT   each block keeps one hot bin (the bin of the first
 *                   in-range voxel it reads) out of LDS and counts it as its
 *                   in-range total minus the other bins: far fewer LDS
 *                   atomics on a skewed histogram, a few more scalar
 *                   instructions per voxel otherwise.
 * Counts are identical in every form.  Histograms of more than 32768 bins
 * use global atomics whatever the form.  Returns the previous form of the
 * thread, or CUBE_EINVAL for an unknown one.
 */
#define CUBE_HIST_AUTO 0
#define CUBE_HIST_PLAIN 1
#define CUBE_HIST_HOT 2
CUBE_API int cube_set_hist_mode(int32_t mode);

/*
 * How the calling thread's later single-box passes (statistics, histogram,
 * fused, the read probe, and the full-box passes of selection, median and
 * quantiles) divide the box among thread blocks.  The two-stage gather of
 * Section 2 leaves the partition of the data open:
 *   CUBE_PARTITION_AUTO (0)    the tuned choice for the pass; without one,
 *                              dynamic for large boxes (chunks of 2^18
 *                              voxels for histogram passes from 2^27 voxels
 *                              on, of 2^19 for statistics passes from 2^30
 *                              on), else static; under an explicit
 *                              cube_set_launch shape, static;
 *   CUBE_PARTITION_STATIC (1)  every block takes one contiguous range of the
 *                              box, fixed at launch;
 *   k in [CUBE_CHUNK_LOG2_MIN, CUBE_CHUNK_LOG2_MAX]
 *                              dynamic: the box is cut into chunks of about
 *                              2^k voxels (at most 65536 chunks) and one
 *                              resident wave of blocks claims them from a
 *                              counter, so that faster parts of the chip take
 *                              more of the box.
 * A dynamic partition keeps one record per chunk, merged in chunk order in
 * FP64, so its results depend on k and the block shape but not on which
 * block took which chunk.  It applies to CUBE_ACCUM_FP64MERGE and to the
 * plain histogram form; other passes keep the static partition.  Counts,
 * selections, medians and quantiles are identical under every partition;
 * the moments differ only in rounding.  Selection passes follow the same
 * automatic rule as histogram passes (chunks of 2^18 voxels from 2^27).
 * Returns the thread's previous setting (0, 1 or k), or CUBE_EINVAL for a
 * value outside these.
 */
#define CUBE_PARTITION_AUTO 0
#define CUBE_PARTITION_STATIC 1
#define CUBE_CHUNK_LOG2_MIN 12
#define CUBE_CHUNK_LOG2_MAX 26
CUBE_API int cube_set_partition(int32_t chunk_log2);

/*
 * The launch plan the calling thread's next single-box pass of kind
 * CUBE_Q_STATS, CUBE_Q_HIST or CUBE_Q_FUSED (nbins bins) over the given
 * DEVICE box would use, as one JSON object written to `out` (at most `cap`
 * bytes, NUL-terminated): threads per block, blocks, float4 loads per tile,
 * LDS histogram copies, histogram form ("none", "lds", "hot", "global"),
 * partition ("static" or "dynamic"), chunk count (0 when static) and work
 * units.  Launches nothing.  Errors: CUBE_EINVAL for the box errors of the
 * other calls, an unknown kind, nbins outside [1, CUBE_MAX_BINS], a NULL
 * `out` or a `cap` too small for the text; CUBE_EDEVICE for a HIP error.
 */
CUBE_API int cube_describe_plan(const float *ptr, const int64_t *dims, int32_t kind,
                                int32_t nbins, char *out, size_t cap);

/*
 * Exact selection and median (Section 3 names the median as a global,
 * multi-pass task).  cube_select stores in *value the valid voxel of rank
 * `rank` (0-based) in the order by value with -0 before +0; CUBE_EINVAL if
 * rank >= n_valid.  cube_median stores the median of the valid voxels: the
 * middle one for odd n_valid, the FP64 mean of the two middle ones for even
 * n_valid (and n_valid in *n_valid when not NULL); CUBE_EINVAL when no voxel
 * is valid.  Three histogram passes over 32-bit order keys (12 + 12 + 8
 * bits), with the bucket choice made on the device; the second pass copies
 * the first pass's bucket out when it fits (64 MiB of device memory kept by
 * the library), and the third then reads only that; for an even count the
 * upper middle comes from the same passes or from at most one more
 * (minimum) pass.  Synchronous, on the default stream; results are exact.
 */
CUBE_API int cube_select(const float *ptr, const int64_t *dims, uint64_t rank, float *value);
CUBE_API int cube_median(const float *ptr, const int64_t *dims, double *median,
                         uint64_t *n_valid);

/*
 * Quantiles of the valid voxels of a DEVICE box at m levels q[0..m-1]
 * (host array, each in [0, 1]; 1 <= m <= CUBE_MAX_QUANTILES).  With n the
 * number of valid voxels, level q takes h = q (n - 1) in FP64, j = floor(h),
 * f = h - j, the valid voxels a and b of ranks j and j + 1 (b = a when
 * f == 0; ranks in the order by value with -0 before +0) and gives
 * a + f (b - a) in FP64: the linear-interpolation quantile (Hyndman and
 * Fan's definition 7), so q = 0 and 1 give the minimum and maximum.  When
 * a == b the result is a; an infinite end point is the result (a = -Inf or
 * b = +Inf) and -Inf to +Inf gives NaN.  At q = 1/2 this is the median up to
 * rounding: cube_median averages (a + b) / 2 instead.
 * Results go to out[0..m-1] (host), the valid count to *n_valid (host; may
 * be NULL).  Three reads of the box when the ranks wanted (two per level at
 * most) fall in at most eight distinct leading 12-bit key buckets and number
 * at most 96, four otherwise; synchronous on the null stream.  Keeps about 300 KB of device and
 * pinned host memory per device until cube_shutdown.  Errors: CUBE_EINVAL
 * for the box errors of the other calls, an empty box, no valid voxel (with
 * *n_valid = 0), NULL q or out, m outside its range or a level outside
 * [0, 1] (NaN included); CUBE_EDEVICE for a HIP error.
 */
#define CUBE_MAX_QUANTILES 64
CUBE_API int cube_quantiles(const float *ptr, const int64_t *dims, const double *q, int32_t m,
                            double *out, uint64_t *n_valid);

/*
 * Number of reads of the box (3 or 4, see cube_quantiles) that the CALLING
 * THREAD's last successful cube_quantiles call made, for measuring its bytes
 * moved; 0 before the thread's first successful call.  Never fails.
 */
CUBE_API int cube_last_quantile_reads(void);

/*
 * Projections along the channel axis z: the maps a viewer of spectral cubes
 * shows beside the rendered volume (Section 2).  For every spatial pixel
 * (x, y) of the box, over its nz channels:
 *   mip[x + nx*y]     float    the maximum valid voxel (-0 < +0); NaN if none
 *   mom0[x + nx*y]    double   the sum of the valid voxels over the extended
 *                              reals (+Inf and -Inf together give NaN); NaN
 *                              if none.  Times the channel width it is the
 *                              moment-0 map.
 *   nvalid[x + nx*y]  uint32   the number of valid channels
 * The outputs are dense DEVICE arrays of nx*ny elements; any may be NULL but
 * not all three.  Stream-ordered on `stream` (NULL = the default stream).
 * Sums are FP64 in channel order within each of at most 64 channel slices,
 * the slices merged in order; results depend only on the shape.  nz == 0
 * gives NaN / NaN / 0 maps.  Errors: CUBE_EINVAL for the box errors of the
 * other calls, outputs that are not device memory of the needed size or are
 * misaligned (mom0 8-byte), or nz >= 2^32; CUBE_EDEVICE for a HIP error.
 */
CUBE_API int cube_project(const float *ptr, const int64_t *dims, float *mip, double *mom0,
                          uint32_t *nvalid, void *stream);

/*
 * Read probe: the read ceiling of the fused pass's access pattern, the
 * figure the fused pass's HBM rate is measured against.  Reads every voxel of
 * the DEVICE box once, in the launch shape the fused statistics-and-histogram
 * pass would use for `nbins` bins (grid, block size, dynamic LDS, tiles per
 * lane, work units per block), doing one bitwise OR per voxel.  ORs the bit
 * patterns of all voxels (NaNs included) into *dev_out, a 4-byte-aligned
 * DEVICE word that the caller zeroes beforehand; the box's own OR is
 * therefore known exactly.  Stream-ordered on `stream` (NULL = the default
 * stream); an empty box launches nothing.  Errors: CUBE_EINVAL for the box
 * errors of the other calls, nbins outside [1, CUBE_MAX_BINS] or a NULL or
 * misaligned dev_out; CUBE_EDEVICE for a HIP error.
 */
CUBE_API int cube_read_probe(const float *ptr, const int64_t *dims, int32_t nbins,
                             uint32_t *dev_out, void *stream);

/*
 * Autotuner.  Times candidate launch shapes (threads, float4 loads per tile,
 * LDS histogram copies, blocks per CU, the hot-bin histogram form, and the
 * static or a dynamic partition with chunks of 2^18, 2^19 or 2^20 voxels
 * under CUBE_ACCUM_FP64MERGE) of one pass kind -- CUBE_Q_STATS,
 * CUBE_Q_HIST or CUBE_Q_FUSED over [lo, hi] -- on the given DEVICE box
 * (`reps` timed launches each) and keeps the fastest for that pass kind,
 * histogram-size class (bins rounded up to a power of two) and box-size
 * class (voxels rounded up to a power of two).  Later single-box calls
 * without an explicit cube_set_launch shape use it.  If `report` is not
 * NULL, a JSON summary is written there.  Results never depend on the shape
 * except for the rounding of the moments.
 */
CUBE_API int cube_autotune(const float *ptr, const int64_t *dims, int32_t kind, float lo,
                           float hi, int32_t nbins, int32_t reps, char *report, size_t report_cap);
/* Save / load the tuned table (JSON, one entry per line, arch "gfx950");
 * load returns the number of entries read. */
CUBE_API int cube_tune_save(const char *path);
CUBE_API int cube_tune_load(const char *path);
CUBE_API void cube_tune_clear(void);

/* Release every workspace on every device (waiting for the last work queued
 * with each).  The library stays usable; workspaces are made again on demand. */
CUBE_API void cube_shutdown(void);

/* The single-box calls keep one workspace (about 2 MiB of device and pinned
 * memory) per (device, stream) they were given, until cube_shutdown.  Call
 * this before destroying a stream that was passed to them: it waits for the
 * stream's last call and frees its workspaces (a later call on the same
 * stream makes a new one).  Not concurrently with calls on that stream.  A
 * stream handle that is destroyed and then reused by a new stream must be
 * released in between, or the new stream inherits the old one's workspace.
 * NULL is the default stream.  Never fails. */
CUBE_API void cube_release_stream(void *stream);

/* ------------------------------------------------------------------------
 * Batched queries in one persistent launch (the paper's batched analysis
 * service, Abstract; many sub-cubes of one dataset, Section 3).
 * ------------------------------------------------------------------------ */

#define CUBE_Q_STATS 0  /* statistics                                       */
#define CUBE_Q_HIST 1   /* histogram over [lo, hi]                           */
#define CUBE_Q_FUSED 2  /* statistics + histogram over [lo, hi], one read   */
#define CUBE_Q_MINMAX 3 /* statistics, then histogram over the box's [min, max] */

typedef struct cube_query_t {
    const float *ptr;   /* DEVICE data, 4-byte aligned (same rules as above) */
    int64_t dims[5];    /* nx, ny, nz, sy, sz (0 pitch = dense)              */
    int32_t kind;       /* CUBE_Q_*                                          */
    int32_t nbins;      /* histogram kinds: 1..32768                         */
    float lo, hi;       /* CUBE_Q_HIST, CUBE_Q_FUSED                         */
    cube_stats_t *out;  /* DEVICE, one cube_stats_t (kinds with statistics)  */
    uint64_t *counts;   /* DEVICE, nbins + 3 (kinds with a histogram)        */
} cube_query_t;

/* An opaque batch: device work-list buffers, grown on demand and reused.
 * One batch runs one work list at a time; use several batches (one per
 * stream) to overlap batches on the device. */
typedef struct cube_batch cube_batch_t;

CUBE_API int cube_batch_create(cube_batch_t **out);
/* Waits for the batch's last launch, then frees everything. */
CUBE_API void cube_batch_destroy(cube_batch_t *b);
/* Tile size in voxels (4096..2^30; default 2^20; 0 = automatic per query)
 * and threads per block (0 = automatic) for later enqueues.  The automatic
 * size comes from the query's voxel count by the batched launch's rule (the
 * tuned one, else the default: the smallest power of two from 2^17 to 2^20
 * that cuts the query into at most 1024 tiles), so it depends on the query
 * alone.  A query's
 * results depend only on its own data and its tile size, not on the other
 * queries of the batch. */
CUBE_API int cube_batch_set_tile(cube_batch_t *b, int64_t tile_voxels, int32_t threads);
/* Validate the n queries (every check of the single-box calls, on the
 * host), build the work list, copy it to the device and launch, all on
 * `stream` (a hipStream_t).  Results are valid when the stream reaches this
 * point.  Each query's results are the same as those of the matching
 * single-box call, except for the rounding of mean and m2 (the tiling
 * differs); counts and extrema are bit-exact. */
CUBE_API int cube_batch_enqueue(cube_batch_t *b, const cube_query_t *q, int32_t n, void *stream);
/* Order of the queries' tiles in the work list: largest queries first (the
 * default; shortest batch) or smallest first (lowest latency for small
 * queries, whose completion is visible as soon as their tiles are done). */
#define CUBE_ORDER_LARGEST_FIRST 0
#define CUBE_ORDER_SMALLEST_FIRST 1
CUBE_API int cube_batch_set_order(cube_batch_t *b, int32_t order);
/* 1 when query i of the last launch of b has completed (its device outputs
 * are final), 0 while it has not, and CUBE_EDEVICE when it completed as
 * failed: a two-pass query whose bounded wait for its own [min, max] range
 * expired (its histogram is then incomplete; other queries are unaffected).
 * Reads a host-mapped flag that the kernel writes, with no GPU call.  Valid
 * after cube_batch_enqueue and cube_batch_relaunch (a graph replay repeats
 * the generation it captured, so use the stream). */
CUBE_API int cube_batch_query_done(cube_batch_t *b, int32_t i);
/* Launch the last enqueued work list again (no host work, no copies).
 * Launches of one batch object are ordered: one on another stream than the
 * previous launch waits, on the device, for that launch to finish. */
CUBE_API int cube_batch_relaunch(cube_batch_t *b, void *stream);
/* Same as cube_batch_relaunch through a captured HIP graph: the first call
 * after an enqueue captures the launch, later calls replay it on any stream. */
CUBE_API int cube_batch_graph_launch(cube_batch_t *b, void *stream);
/* Wait for the batch and report whether every two-pass query of the
 * launches since the last check completed: CUBE_EDEVICE if a query's bounded
 * wait for its range expired (reported once; the flag is then cleared).
 * A range published by one launch never releases the second phase of a
 * later launch, so the launches after a failure run normally.  Test knob:
 * CUBE_FAULT_INJECT="expire:N[,M...]" (read by cube_batch_create): in the
 * batch's launches N, M, ... (counted from 1 over enqueues and relaunches;
 * graph replays excluded) every range wait gives up at once. */
CUBE_API int cube_batch_check(cube_batch_t *b);
/* Synchronous convenience: create, enqueue on the default stream, check,
 * destroy. */
CUBE_API int cube_batch_run(const cube_query_t *q, int32_t n);

/*
 * Autotuner of the batched launch.  Times candidate automatic rules -- threads
 * per block (256 or 512: 1024-thread blocks leave no room on a CU for a
 * concurrent batch), float4 loads per lane per pipelined step (2
 * or 4), each query's tile size as a function of its
 * own voxel count (a floor of 2^16..2^18 voxels, doubled up to a cap of
 * 2^19..2^21 while the query needs more than 2^8..2^10 tiles) and the LDS
 * budget of the histogram copies (64 or 128 KiB) -- as graph-replayed
 * launches of a batch of the caller's n queries (`reps` timed replays each;
 * the queries' device outputs are overwritten), and keeps the fastest as the
 * rule for every later batch whose tile size and threads are automatic
 * (cube_batch_set_tile(b, 0, 0); the server's default).  One rule serves all
 * batches, so a query's tiling depends on the query alone.  The rule is
 * saved and loaded with the tuning table.  If `report` is not NULL, a JSON
 * summary is written there.  Errors: those of cube_batch_enqueue; CUBE_EINVAL
 * for n < 1 or reps outside [1, 100].
 */
CUBE_API int cube_autotune_batch(const cube_query_t *q, int32_t n, int32_t reps, char *report,
                                 size_t report_cap);


/*
 * Out-of-core query over a cube in HOST memory.  The paper's cubes exceed
 * one device and are processed as sub-cubes while loading overlaps
 * processing (Sections 2 and 3).  `q->ptr` is host memory: pinned memory
 * (hipHostMalloc) is copied by the DMA engine directly; pageable memory is
 * gathered by a few host threads into three pinned 64 MiB staging buffers
 * (kept until cube_shutdown) while the previous chunk is copied, in chunks
 * of at most 2^24 voxels.  `q->out` (cube_stats_t) and
 * `q->counts` (nbins + 3 uint64) are HOST outputs; `q->kind`, `dims`, `lo`,
 * `hi` and `nbins` mean what they mean for the resident calls.  The box is
 * cut into chunks of at most `chunk_voxels` voxels (0 = 2^28; allowed
 * [2^12, 2^31]), runs of whole rows of one plane, each copied by a copy
 * stream into one of three device buffers while the previous chunk is
 * processed.  Counts are exact and equal the resident results; statistics
 * merge the chunks' records in chunk order in FP64 and agree with the
 * resident results within the moment tolerance.  CUBE_Q_MINMAX reads the
 * host cube twice.  Synchronous; the library keeps 3 x chunk_voxels x 4
 * bytes of device memory for later calls (released by cube_shutdown).
 * Errors: CUBE_EINVAL for a device pointer or the resident calls' argument
 * errors, CUBE_EDEVICE for a HIP error; calls on one device are serialised.
 */
CUBE_API int cube_host_query(const cube_query_t *q, int64_t chunk_voxels);

/* ------------------------------------------------------------------------
 * Query server over cubes resident in GPU memory (the paper's analysis as a
 * service for many users, with batched and real-time requests: Abstract,
 * Sections 2 and 3).  Continuous batching: a worker thread forms batches of
 * waiting queries whenever one of `slots` streams is free and the device
 * scratch in flight stays within `max_inflight_bytes`, and launches each
 * batch as one persistent launch, so batches overlap on the device.
 * CUBE_SERVE_PLAIN instead runs one query at a time, in arrival order,
 * through the single-box entry points (the baseline).
 * ------------------------------------------------------------------------ */

#define CUBE_SERVE_BATCHED 0
#define CUBE_SERVE_PLAIN 1

typedef struct cube_server cube_server_t;

/* slots: 1..16 concurrent batches; max_batch: queries per batch (1..4096);
 * max_inflight_bytes: device scratch budget (>= 4096); tile_voxels: 0 =
 * each query's automatic size (see cube_batch_set_tile), else 4096..2^30.  The calling thread's current device is used.
 * A batch whose launch fails, or whose completion event reports a device
 * error, completes its unfinished queries with CUBE_EDEVICE and frees its
 * slot; a two-pass query whose range wait expired completes with
 * CUBE_EDEVICE alone.  The server goes on serving either way.  Failure
 * handling can be tested with the environment variable CUBE_FAULT_INJECT
 * (read at creation; launches counted from 1 per server): "launch:N[,M...]"
 * fails launches N, M, ... on the host before any work is queued;
 * "event:N" makes the completion event of launch N report an error (the
 * work itself runs to its end); "expire:N" reaches the slots' batches
 * (see cube_batch_check).  Items combine: "launch:2,event:4,expire:1". */
CUBE_API int cube_server_create(int32_t mode, int32_t slots, int32_t max_batch,
                                int64_t max_inflight_bytes, int64_t tile_voxels,
                                cube_server_t **out);
/* Queue one query (host-side checks now; CUBE_EBUSY when the queue is full).
 * The query's device outputs must stay valid until it completes.  Returns
 * its id in *id.  Thread-safe. */
CUBE_API int cube_server_submit(cube_server_t *s, const cube_query_t *q, uint64_t *id);
/* Wait up to timeout_s (< 0: no limit) for query `id`; on completion its
 * outputs are valid, the latency from submission to completion is stored
 * in *latency_s, and the id is retired.  CUBE_EBUSY on timeout (the id stays
 * valid); the query's own error code if it failed. */
CUBE_API int cube_server_wait(cube_server_t *s, uint64_t id, double timeout_s, double *latency_s);
/* Latency percentiles (seconds) over the queries completed so far;
 * `reset` != 0 clears the record. */
CUBE_API int cube_server_latency(cube_server_t *s, double *p50_s, double *p99_s,
                                 uint64_t *n_done, int32_t reset);
/* Finish the queued and running queries, then stop and free the server. */
CUBE_API void cube_server_destroy(cube_server_t *s);

#ifdef __cplusplus
}
#endif

#endif /* CUBESTATS_H */
