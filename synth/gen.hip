// gen.hip -- seeded synthetic spectral-cube generator (input generator only).
//
// This module makes test and benchmark inputs.  It holds none of the
// statistics or histogram arithmetic, and neither the oracle nor the GPU
// statistics library includes or links it: both only read the float32 bytes it
// writes.
//
// A voxel (x, y, z) of the box at p[x + sy*y + sz*z] receives
//     offset + noise_sigma * N(0,1)
//   + sum over the sources listed for its tile, in source order, of
//     A_s * exp(-0.5 * ((x-cx)^2/sx^2 + (y-cy)^2/sy^2 + (z-cz)^2/sz^2))
//     for |x-cx| <= rx, |y-cy| <= ry, |z-cz| <= rz (truncated footprint),
// evaluated in FP64 and rounded once to float32, and is then blanked (NaN) if
//   - a per-voxel Bernoulli draw falls under p_voxel_nan, or
//   - its spatial pixel (x, y) is blanked (per-pixel draw under p_pixel_nan), or
//   - its channel z lies in one of the blanked channel ranges.
//
// Random numbers come from SplitMix64 (Steele, Lea & Flood 2014) used as a
// counter-based hash of (seed, stream, index); normals from the Box-Muller
// transform.  The sources (centres, amplitudes) are drawn on the host and
// binned into tiles of TILE^3 voxels so that every voxel sums the sources of
// its own tile in a fixed order: the output is the same on every run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SYNTH_TILE 32

struct synth_recipe_t {
    uint64_t seed;
    int64_t nx, ny, nz, sy, sz;
    double offset, noise_sigma;
    double sig_x, sig_y, sig_z;
    int32_t rad_x, rad_y, rad_z, n_chan_ranges;
    double p_voxel_nan, p_pixel_nan;
    int32_t chan_lo[8], chan_hi[8];
    // Sources: centre (cx, cy, cz) and amplitude, device arrays of n_sources.
    const double *src;           // [n_sources][4] = cx, cy, cz, amp
    int64_t n_sources;
    // Tile lists: tile t holds src_idx[tile_start[t] .. tile_start[t+1]).
    const int32_t *tile_start;   // n_tiles + 1 entries
    const int32_t *src_idx;
    int64_t tiles_x, tiles_y, tiles_z;
};

__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Hash of (seed, stream, index): two rounds so that neighbouring indices and
// streams decorrelate.
__device__ __forceinline__ uint64_t hash3(uint64_t seed, uint64_t stream, uint64_t idx)
{
    return splitmix64(splitmix64(seed ^ (stream * 0xD1B54A32D192ED03ull)) + idx);
}

__device__ __forceinline__ double unit_open(uint64_t h)   // (0, 1)
{
    return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

__global__ void __launch_bounds__(256)
synth_fill(synth_recipe_t r, float *__restrict__ p)
{
    const int64_t n = r.nx * r.ny * r.nz;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += step) {
        const int64_t x = v % r.nx;
        const int64_t t = v / r.nx;
        const int64_t y = t % r.ny;
        const int64_t z = t / r.ny;

        // Noise.
        const double u1 = unit_open(hash3(r.seed, 1, (uint64_t)v));
        const double u2 = unit_open(hash3(r.seed, 2, (uint64_t)v));
        double val = r.offset
                   + r.noise_sigma * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);

        // Sources of this voxel's tile, in source order.
        const int64_t tx = x / SYNTH_TILE, ty = y / SYNTH_TILE, tz = z / SYNTH_TILE;
        const int64_t tile = tx + r.tiles_x * (ty + r.tiles_y * tz);
        const int32_t s0 = r.tile_start[tile], s1 = r.tile_start[tile + 1];
        for (int32_t k = s0; k < s1; ++k) {
            const double *s = r.src + 4 * (int64_t)r.src_idx[k];
            const double dx = (double)x - s[0], dy = (double)y - s[1], dz = (double)z - s[2];
            if (fabs(dx) > r.rad_x || fabs(dy) > r.rad_y || fabs(dz) > r.rad_z) continue;
            const double q = dx * dx / (r.sig_x * r.sig_x) + dy * dy / (r.sig_y * r.sig_y)
                           + dz * dz / (r.sig_z * r.sig_z);
            val += s[3] * exp(-0.5 * q);
        }
        float out = (float)val;

        // Blanking, written last.
        bool blank = false;
        if (r.p_voxel_nan > 0.0 && unit_open(hash3(r.seed, 3, (uint64_t)v)) < r.p_voxel_nan)
            blank = true;
        if (r.p_pixel_nan > 0.0 &&
            unit_open(hash3(r.seed, 4, (uint64_t)(x + r.nx * y))) < r.p_pixel_nan)
            blank = true;
        for (int i = 0; i < r.n_chan_ranges; ++i)
            if (z >= r.chan_lo[i] && z < r.chan_hi[i]) blank = true;
        if (blank) out = __int_as_float(0x7fc00000);

        p[x + r.sy * y + r.sz * z] = out;
    }
}

extern "C" {

// Fill the box at device pointer p (float32, pitches sy, sz in elements).
// Returns 0, or the HIP error code of the launch.
int synth_fill_box(const synth_recipe_t *r, float *p, void *stream)
{
    const int64_t n = r->nx * r->ny * r->nz;
    if (n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(synth_fill, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, *r, p);
    return (int)hipGetLastError();
}

int synth_recipe_size(void) { return (int)sizeof(synth_recipe_t); }
int synth_tile(void) { return SYNTH_TILE; }

}
