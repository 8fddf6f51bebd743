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
int cube_abi_version(void);

/* Text of the calling thread's last error ("" if none).  Valid until the next
 * call from the same thread. */
const char *cube_last_error(void);

/*
 * Statistics of one box in one pass (Abstract: data minimum/maximum;
 * Section 3: standard deviation).  `stride` is NULL (dense) or a HOST array
 * {sy, sz} of pitches in elements.  `out` is HOST memory.  Synchronous.
 */
int cube_stats(const float *ptr, int64_t nx, int64_t ny, int64_t nz,
               const int64_t *stride, cube_stats_t *out);

/*
 * Histogram of one box over a given range (Abstract: the histogram task).
 * `counts` is HOST memory of nbins + 3 uint64.  Synchronous.
 */
int cube_hist(const float *ptr, const int64_t *dims, float lo, float hi,
              int32_t nbins, uint64_t *counts);

/*
 * Statistics and the histogram over a given range in ONE launch reading each
 * voxel once.  Results equal those of cube_stats and cube_hist (counts and
 * extrema bit-exact; moments within rounding).  HOST outputs.  Synchronous.
 */
int cube_stats_hist(const float *ptr, const int64_t *dims, float lo, float hi,
                    int32_t nbins, cube_stats_t *out, uint64_t *counts);

/*
 * Two passes: statistics, then the histogram over the data's own range
 * [min, max] (the range and its FP32 scale are formed on the device, so the
 * host never waits between the passes).  With no valid voxel the bins are 0
 * and the NaN counter holds n_total; with an invalid [min, max] range (see
 * CUBE_HIST_BAD_RANGE) the statistics are returned, the bins are 0, and the
 * call returns CUBE_EINVAL.  HOST outputs.  Synchronous.
 */
int cube_stats_hist_minmax(const float *ptr, const int64_t *dims, int32_t nbins,
                           cube_stats_t *out, uint64_t *counts);

/* Stream-ordered forms of the four calls above.  `dev_out` (one
 * cube_stats_t) and `dev_counts` (nbins + 3 uint64) are DEVICE memory. */
int cube_stats_async(const float *ptr, const int64_t *dims, cube_stats_t *dev_out,
                     void *stream);
int cube_hist_async(const float *ptr, const int64_t *dims, float lo, float hi,
                    int32_t nbins, uint64_t *dev_counts, void *stream);
int cube_stats_hist_async(const float *ptr, const int64_t *dims, float lo,
                          float hi, int32_t nbins, cube_stats_t *dev_out,
                          uint64_t *dev_counts, void *stream);
int cube_stats_hist_minmax_async(const float *ptr, const int64_t *dims,
                                 int32_t nbins, cube_stats_t *dev_out,
                                 uint64_t *dev_counts, void *stream);

/*
 * Precision mode of the moments for later calls from any thread (the
 * FP32-only modes exist to compare against; only CUBE_ACCUM_FP64MERGE meets
 * the 1e-6 relative bound on hard inputs).  Returns the previous mode, or
 * CUBE_EINVAL for an unknown mode.
 */
int cube_set_accum_mode(int32_t mode);

/*
 * Launch-shape override for the single-box calls, used by the autotuner and
 * for experiments: threads per block (256, 512 or 1024; 0 = automatic),
 * blocks per launch (0 = automatic), histogram sub-copies per block (1..32,
 * a power of two; 0 = automatic).  Applies to later calls from any thread.
 */
int cube_set_launch(int32_t threads, int32_t blocks, int32_t hist_copies);

/* Release every workspace on every device (synchronises each stream that
 * owns one).  The library stays usable; workspaces are made again on demand. */
void cube_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* CUBESTATS_H */
