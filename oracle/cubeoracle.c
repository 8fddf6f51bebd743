/*
 * cubeoracle.c -- the CPU oracle for the cube statistics + histogram pass.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library.  It shares
 * no source, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * What it computes.  Hassan, Fluke & Barnes name the data-analysis tasks their
 * framework serves on a spectral cube: the data minimum and maximum and a
 * histogram (Abstract), and the standard deviation (Section 3, where it is
 * given as an example of a global, multi-pass task).  The paper fixes none of
 * the arithmetic, so every result here is the plain mathematical definition,
 * written out in the most direct way, in double precision:
 *
 *   blank voxel  : a NaN of any bit pattern (tested by x != x).  +-Inf are
 *                  ordinary values.
 *   n_total      : nx * ny * nz
 *   n_nan        : number of blank voxels; n_valid = n_total - n_nan
 *   min, max     : over valid voxels, ordered by value with -0 < +0
 *   mean         : (1/n_valid) * sum x                      over valid voxels
 *   m2           : sum (x - mean)^2                         over valid voxels
 *   std          : sqrt(m2 / n_valid)   (population standard deviation)
 *   mean_abs     : (1/n_valid) * sum |x|  (only used to scale tolerances)
 *
 *   These sums are taken over the extended reals, as IEEE arithmetic defines
 *   them for +-Inf, not as a rounding artifact of any summation order: with
 *   +Inf among the valid voxels (and no -Inf) the mean is +Inf, with -Inf
 *   alone it is -Inf, with both it is NaN (Inf - Inf); mean_abs is then +Inf;
 *   and since some deviation x - mean is then Inf - Inf or an infinite mean
 *   minus a finite x, m2 and std are NaN.  The finite voxels are summed
 *   apart from the infinities so that the finite case is exact as before.
 *
 *   select(k)    : the valid voxel of rank k (0-based) in the order by value
 *                  with -0 before +0; median = select((n-1)/2) for odd
 *                  n_valid, the FP64 mean of select(n/2-1) and select(n/2)
 *                  for even n_valid (the median task of Section 3).
 *   quantile(q)  : for 0 <= q <= 1, with n = n_valid, h = q * (n - 1) in FP64,
 *                  j = floor(h), f = h - j, a = select(j) and b = select(j+1)
 *                  (b = a when f == 0): the linear interpolation a + f*(b - a)
 *                  in FP64 (Hyndman and Fan's definition 7, numpy's default).
 *                  When a == b the result is a; an infinite end point is the
 *                  result (a = -Inf or b = +Inf), and -Inf to +Inf gives NaN.
 *
 *   projections along the channel axis, per spatial pixel (x, y) over the
 *   channels z of the box (the maps shown beside a rendered cube):
 *      mip(x, y)    : the maximum valid voxel (-0 < +0), NaN when none
 *      mom0(x, y)   : the sum of the valid voxels (FP64, over the extended
 *                     reals: +Inf and -Inf together give NaN), NaN when none
 *      nvalid(x, y) : the number of valid voxels
 *
 *   histogram over a closed range [lo, hi] with nbins bins, decided in FP32:
 *      blank            -> the NaN counter
 *      x < lo           -> the "below" counter
 *      x > hi           -> the "above" counter
 *      otherwise        -> bin min(nbins - 1, floor((x - lo) * scale)),
 *                          scale = (float)nbins / (hi - lo), every operation a
 *                          single rounded FP32 operation in exactly this order;
 *                          if hi == lo every in-range voxel (x == lo) is bin 0.
 *
 * Sums use Neumaier's compensated summation (Neumaier 1974) in FP64; m2 uses
 * the corrected two-pass form m2 = sum d^2 - (sum d)^2 / n with d = x - mean
 * (Chan, Golub & LeVeque 1983).  Both only refine the rounding of the plain
 * definition; neither changes what is computed.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * No FMA contraction and no flush-to-zero: on x86-64 every float and double
 * operation is a single IEEE round-to-nearest-even operation.
 *
 * Layout: voxel (x, y, z) of a box lives at p[x + sy*y + sz*z], x fastest and
 * the channel axis z slowest; a dense cube has sy = nx, sz = nx*ny.
 *
 * Every entry point can be called repeatedly on pieces of a cube ("chunk
 * streaming") so that a cube larger than host memory can be checked piece by
 * piece: sweep 1 over all pieces, then sweep 2 over all pieces, then finish.
 * The sweep records of separate slabs can also be added together in slab
 * order (oracle_sweep*_add), so that slabs are swept on several threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#if defined(__FAST_MATH__)
#error "the oracle must not be built with fast-math"
#endif

#define ORACLE_ABI 2

typedef struct {
    uint64_t n_total, n_valid, n_nan;
    float min, max;
    double sum, sum_c;   /* Neumaier pair for sum x   */
    double sabs, sabs_c; /* Neumaier pair for sum |x| */
    uint64_t n_pinf, n_ninf; /* valid voxels equal to +Inf and to -Inf */
} oracle_sweep1_t;

typedef struct {
    uint64_t n;          /* valid voxels seen in sweep 2 */
    double dev, dev_c;   /* Neumaier pair for sum (x - mean)   */
    double sq, sq_c;     /* Neumaier pair for sum (x - mean)^2 */
} oracle_sweep2_t;

typedef struct {
    uint64_t n_total, n_valid, n_nan;
    float min, max;
    double mean, m2, std, mean_abs;
} oracle_stats_t;

int oracle_abi_version(void) { return ORACLE_ABI; }

/* Neumaier's improved Kahan summation: s + c carries the running sum. */
static void neumaier_add(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/* Total order used for min/max: by value, and -0 before +0. */
static int before(float a, float b)
{
    if (a < b) return 1;
    if (a == b && signbit(a) && !signbit(b)) return 1;
    return 0;
}

/* A box is legal when no two voxels share an address: rows do not overlap
 * (sy >= nx when there is more than one row) and planes do not overlap
 * (sz >= sy*(ny-1) + nx when there is more than one plane). */
static int dims_ok(int64_t nx, int64_t ny, int64_t nz, int64_t sy, int64_t sz)
{
    if (nx < 0 || ny < 0 || nz < 0) return 0;
    if (nx == 0 || ny == 0 || nz == 0) return 1;
    if (ny > 1 && sy < nx) return 0;
    if (nz > 1 && sz < (ny - 1) * (ny > 1 ? sy : 0) + nx) return 0;
    return 1;
}

void oracle_sweep1_init(oracle_sweep1_t *s)
{
    memset(s, 0, sizeof *s);
    s->min = NAN;
    s->max = NAN;
}

/* Sweep 1 over one box: counts, extrema, sum x and sum |x|. */
int oracle_sweep1(oracle_sweep1_t *s, const float *p, int64_t nx, int64_t ny,
                  int64_t nz, int64_t sy, int64_t sz)
{
    if (!dims_ok(nx, ny, nz, sy, sz)) return -1;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                float v = p[x + sy * y + sz * z];
                s->n_total++;
                if (v != v) {
                    s->n_nan++;
                    continue;
                }
                if (s->n_valid == 0) {
                    s->min = v;
                    s->max = v;
                } else {
                    if (before(v, s->min)) s->min = v;
                    if (before(s->max, v)) s->max = v;
                }
                s->n_valid++;
                if (isinf(v)) {
                    /* kept apart: the sum of the finite voxels stays finite */
                    if (v > 0) s->n_pinf++; else s->n_ninf++;
                    continue;
                }
                neumaier_add(&s->sum, &s->sum_c, (double)v);
                neumaier_add(&s->sabs, &s->sabs_c, fabs((double)v));
            }
    return 0;
}

/* The mean that sweep 2 needs, from a finished sweep 1 (extended reals:
 * +Inf, -Inf or NaN when infinite voxels are present). */
double oracle_sweep1_mean(const oracle_sweep1_t *s)
{
    if (s->n_valid == 0) return NAN;
    if (s->n_pinf && s->n_ninf) return NAN;
    if (s->n_pinf) return INFINITY;
    if (s->n_ninf) return -INFINITY;
    return (s->sum + s->sum_c) / (double)s->n_valid;
}

void oracle_sweep2_init(oracle_sweep2_t *s) { memset(s, 0, sizeof *s); }

/* Sweep 2 over one box: sum (x - mean) and sum (x - mean)^2. */
int oracle_sweep2(oracle_sweep2_t *s, const float *p, int64_t nx, int64_t ny,
                  int64_t nz, int64_t sy, int64_t sz, double mean)
{
    if (!dims_ok(nx, ny, nz, sy, sz)) return -1;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                float v = p[x + sy * y + sz * z];
                if (v != v) continue;
                double d = (double)v - mean;
                s->n++;
                neumaier_add(&s->dev, &s->dev_c, d);
                neumaier_add(&s->sq, &s->sq_c, d * d);
            }
    return 0;
}

/*
 * Sweep records of consecutive slabs of one cube, added together: a sweep
 * over slab A then slab B in one record equals the record of A with the
 * record of B added by these functions (counts add, extrema by the same
 * order, each compensated sum adds the other's pair).  They let slabs be
 * swept side by side on several host threads and combined in slab order.
 */
void oracle_sweep1_add(oracle_sweep1_t *a, const oracle_sweep1_t *b)
{
    if (b->n_valid) {
        if (a->n_valid == 0) {
            a->min = b->min;
            a->max = b->max;
        } else {
            if (before(b->min, a->min)) a->min = b->min;
            if (before(a->max, b->max)) a->max = b->max;
        }
    }
    a->n_total += b->n_total;
    a->n_valid += b->n_valid;
    a->n_nan += b->n_nan;
    neumaier_add(&a->sum, &a->sum_c, b->sum);
    a->sum_c += b->sum_c;
    neumaier_add(&a->sabs, &a->sabs_c, b->sabs);
    a->sabs_c += b->sabs_c;
    a->n_pinf += b->n_pinf;
    a->n_ninf += b->n_ninf;
}

void oracle_sweep2_add(oracle_sweep2_t *a, const oracle_sweep2_t *b)
{
    a->n += b->n;
    neumaier_add(&a->dev, &a->dev_c, b->dev);
    a->dev_c += b->dev_c;
    neumaier_add(&a->sq, &a->sq_c, b->sq);
    a->sq_c += b->sq_c;
}

void oracle_finish(const oracle_sweep1_t *a, const oracle_sweep2_t *b,
                   oracle_stats_t *out)
{
    out->n_total = a->n_total;
    out->n_valid = a->n_valid;
    out->n_nan = a->n_nan;
    out->min = a->min;
    out->max = a->max;
    if (a->n_valid == 0) {
        out->mean = out->m2 = out->std = out->mean_abs = NAN;
        return;
    }
    double n = (double)a->n_valid;
    out->mean = oracle_sweep1_mean(a);
    if (a->n_pinf || a->n_ninf) {
        /* an infinite voxel: |x| sums to +Inf, and a deviation x - mean is
         * Inf - Inf or infinite, so m2 and std are NaN (extended reals) */
        out->mean_abs = INFINITY;
        out->m2 = out->std = NAN;
        return;
    }
    out->mean_abs = (a->sabs + a->sabs_c) / n;
    double dev = b->dev + b->dev_c;
    double m2 = (b->sq + b->sq_c) - dev * dev / n;
    if (m2 < 0.0) m2 = 0.0; /* only rounding can make it negative */
    out->m2 = m2;
    out->std = sqrt(m2 / n);
}

/* One-shot statistics of one box. */
int oracle_stats(const float *p, int64_t nx, int64_t ny, int64_t nz,
                 int64_t sy, int64_t sz, oracle_stats_t *out)
{
    oracle_sweep1_t a;
    oracle_sweep2_t b;
    oracle_sweep1_init(&a);
    oracle_sweep2_init(&b);
    if (oracle_sweep1(&a, p, nx, ny, nz, sy, sz)) return -1;
    if (oracle_sweep2(&b, p, nx, ny, nz, sy, sz, oracle_sweep1_mean(&a)))
        return -1;
    oracle_finish(&a, &b, out);
    return 0;
}

/*
 * The FP32 scale of the bin formula.  Returns 0 and sets *scale on a valid
 * range; -1 when lo or hi is NaN or infinite, hi < lo, hi - lo overflows, or
 * nbins / (hi - lo) is not finite (a range too narrow for nbins bins), and for
 * nbins outside [1, 65536].
 */
int oracle_hist_scale(float lo, float hi, int32_t nbins, float *scale)
{
    if (nbins < 1 || nbins > 65536) return -1;
    if (!(lo == lo) || !(hi == hi)) return -1;
    if (isinf(lo) || isinf(hi)) return -1;
    if (hi < lo) return -1;
    float width = hi - lo;
    if (isinf(width)) return -1;
    if (width == 0.0f) {
        *scale = 0.0f;
        return 0;
    }
    float s = (float)nbins / width;
    if (isinf(s)) return -1;
    *scale = s;
    return 0;
}

/*
 * Histogram of one box, added onto counts[0 .. nbins+2]: the nbins bins, then
 * below, above and NaN.  The caller zeroes counts once before the first box.
 */
int oracle_hist_accumulate(const float *p, int64_t nx, int64_t ny, int64_t nz,
                           int64_t sy, int64_t sz, float lo, float hi,
                           int32_t nbins, uint64_t *counts)
{
    float scale;
    if (!dims_ok(nx, ny, nz, sy, sz)) return -1;
    if (oracle_hist_scale(lo, hi, nbins, &scale)) return -1;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                float v = p[x + sy * y + sz * z];
                if (v != v) {
                    counts[nbins + 2]++;
                } else if (v < lo) {
                    counts[nbins]++;
                } else if (v > hi) {
                    counts[nbins + 1]++;
                } else {
                    float u = (v - lo) * scale;
                    int64_t b = (int64_t)floorf(u);
                    if (b > nbins - 1) b = nbins - 1;
                    counts[b]++;
                }
            }
    return 0;
}

int oracle_hist(const float *p, int64_t nx, int64_t ny, int64_t nz, int64_t sy,
                int64_t sz, float lo, float hi, int32_t nbins, uint64_t *counts)
{
    if (nbins < 1 || nbins > 65536) return -1;
    memset(counts, 0, sizeof(uint64_t) * (size_t)(nbins + 3));
    return oracle_hist_accumulate(p, nx, ny, nz, sy, sz, lo, hi, nbins, counts);
}

/* qsort comparator for the total order of valid voxels: by value, -0 < +0. */
static int cmp_float(const void *a, const void *b)
{
    float x = *(const float *)a, y = *(const float *)b;
    if (before(x, y)) return -1;
    if (before(y, x)) return 1;
    return 0;
}

/*
 * The valid voxel of rank k (0-based) of one box, by sorting every valid
 * voxel.  Returns 0, or -1 for an invalid box or k >= n_valid, or -2 when
 * the copy cannot be allocated.
 */
int oracle_select(const float *p, int64_t nx, int64_t ny, int64_t nz, int64_t sy,
                  int64_t sz, uint64_t k, float *value)
{
    if (!dims_ok(nx, ny, nz, sy, sz)) return -1;
    uint64_t n = 0, cap = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    float *v = (float *)malloc((cap ? cap : 1) * sizeof(float));
    if (!v) return -2;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                float f = p[x + sy * y + sz * z];
                if (f == f) v[n++] = f;
            }
    if (k >= n) {
        free(v);
        return -1;
    }
    qsort(v, (size_t)n, sizeof(float), cmp_float);
    *value = v[k];
    free(v);
    return 0;
}

/* Median of the valid voxels (see the header); -1 when there is none. */
int oracle_median(const float *p, int64_t nx, int64_t ny, int64_t nz, int64_t sy,
                  int64_t sz, double *median, uint64_t *n_valid)
{
    oracle_stats_t st;
    if (oracle_stats(p, nx, ny, nz, sy, sz, &st)) return -1;
    *n_valid = st.n_valid;
    if (st.n_valid == 0) return -1;
    float a, b;
    if (st.n_valid % 2 == 1) {
        if (oracle_select(p, nx, ny, nz, sy, sz, (st.n_valid - 1) / 2, &a)) return -1;
        *median = (double)a;
    } else {
        if (oracle_select(p, nx, ny, nz, sy, sz, st.n_valid / 2 - 1, &a)) return -1;
        if (oracle_select(p, nx, ny, nz, sy, sz, st.n_valid / 2, &b)) return -1;
        *median = ((double)a + (double)b) / 2.0;
    }
    return 0;
}

/*
 * Quantiles of the valid voxels (see the header): one sort, then for every
 * level q[i] the interpolation between the two valid voxels around rank
 * q[i] * (n - 1).  Returns 0, or -1 for an invalid box, a level outside
 * [0, 1] (NaN included) or no valid voxel, or -2 when the copy cannot be
 * allocated.  *n_valid is set whenever the box is valid.
 */
int oracle_quantiles(const float *p, int64_t nx, int64_t ny, int64_t nz, int64_t sy,
                     int64_t sz, const double *q, int32_t m, double *out, uint64_t *n_valid)
{
    if (!dims_ok(nx, ny, nz, sy, sz) || m < 1) return -1;
    uint64_t n = 0, cap = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    float *v = (float *)malloc((cap ? cap : 1) * sizeof(float));
    if (!v) return -2;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                float w = p[x + sy * y + sz * z];
                if (w != w) continue;  /* blank */
                v[n++] = w;
            }
    *n_valid = n;
    int rc = 0;
    for (int32_t i = 0; i < m; ++i)
        if (!(q[i] >= 0.0 && q[i] <= 1.0)) rc = -1;
    if (n == 0 || rc) {
        free(v);
        return -1;
    }
    qsort(v, (size_t)n, sizeof(float), cmp_float);
    for (int32_t i = 0; i < m; ++i) {
        double h = q[i] * (double)(n - 1);
        double j = floor(h);
        double f = h - j;
        double a = v[(uint64_t)j];
        double b = f > 0.0 ? v[(uint64_t)j + 1] : a;
        double r;
        if (a == b)
            r = a;
        else if (isinf(a) && isinf(b))
            r = NAN;
        else if (isinf(a))
            r = a;
        else if (isinf(b))
            r = b;
        else
            r = a + f * (b - a);
        out[i] = r;
    }
    free(v);
    return 0;
}

/*
 * Projections along the channel axis (see the header): dense nx*ny maps,
 * pixel (x, y) at index x + nx*y; any output may be NULL.  Returns 0, or -1
 * for an invalid box.
 */
int oracle_project(const float *p, int64_t nx, int64_t ny, int64_t nz, int64_t sy,
                   int64_t sz, float *mip, double *mom0, uint32_t *nvalid)
{
    if (!dims_ok(nx, ny, nz, sy, sz)) return -1;
    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            float mx = NAN;
            double s = 0.0, c = 0.0;
            uint32_t n = 0;
            int pinf = 0, ninf = 0;
            for (int64_t z = 0; z < nz; ++z) {
                float f = p[x + sy * y + sz * z];
                if (f != f) continue;
                if (n == 0 || before(mx, f)) mx = f;
                /* the sum over the extended reals: infinities apart */
                if (isinf(f))
                    *(f > 0 ? &pinf : &ninf) = 1;
                else
                    neumaier_add(&s, &c, (double)f);
                ++n;
            }
            double sum = s + c;
            if (pinf || ninf) sum = (pinf && ninf) ? NAN : (pinf ? INFINITY : -INFINITY);
            const int64_t i = x + nx * y;
            if (mip) mip[i] = mx;
            if (mom0) mom0[i] = n ? sum : NAN;
            if (nvalid) nvalid[i] = n;
        }
    return 0;
}
