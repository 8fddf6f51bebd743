"""Seeded synthetic spectral cubes: the inputs of the tests and the benchmark.

This package is an input generator only.  It holds none of the statistics or
histogram arithmetic; the oracle and the GPU library both read the float32
bytes it produces and share nothing else through it.

A cube is i.i.d. Gaussian noise (``offset + noise_sigma * N(0,1)``) plus point
sources, each a separable 3-D Gaussian (sigma 1.5 px spatial, 4 channels
spectral, truncated at 4 sigma) at a continuous uniform random centre, with a
peak amplitude drawn uniform or log-uniform; then blanked voxels (NaN): a
per-voxel Bernoulli fraction, whole spatial pixels blanked over all channels,
and contiguous blanked channel ranges.  The data model follows the spectral
cubes of the paper's case study (Section 2) with the shapes and value
distributions of the workloads listed in ``WORKLOADS``.

Two implementations of the same recipe:
  * ``fill_device`` -- a HIP kernel (``gen.hip``) writing straight into device
    memory; used for every cube the GPU tests and the benchmark touch.
  * ``make_numpy`` -- a numpy version for CPU-only tests of small cubes.
Both hash (seed, stream, index) with SplitMix64 and use Box-Muller, so they
agree to the last bit except where the two math libraries round a log, cos or
exp differently.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.hip")
_LIB = os.path.join(_HERE, "libcubesynth.so")
TILE = 32
BASE_SEED = 11116661

HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build() -> str:
    """Compile the generator for gfx950 (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["hipcc", *HIPCC_FLAGS, "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


@dataclass(frozen=True)
class Recipe:
    """How to build one synthetic cube.  Sizes are (nx, ny, nz) = (x, y, channel)."""
    nx: int
    ny: int
    nz: int
    n_sources: int = 20
    amp_dist: str = "uniform"          # "uniform" or "loguniform"
    amp_lo: float = 5.0
    amp_hi: float = 50.0
    offset: float = 0.0
    noise_sigma: float = 1.0
    sigma: tuple = (1.5, 1.5, 4.0)
    radius: tuple = (6, 6, 16)         # truncation at 4 sigma, in voxels
    p_voxel_nan: float = 0.0           # per-voxel blanking
    p_pixel_nan: float = 0.0           # per spatial pixel, all channels
    chan_nan_frac: float = 0.0         # fraction of channels blanked ...
    chan_nan_ranges: int = 0           # ... as this many contiguous ranges

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def scaled(self, nx: int, ny: int, nz: int, min_sources: int = 1) -> "Recipe":
        """Same recipe at another size, with the source count scaled by volume."""
        k = (nx * ny * nz) / self.n
        return replace(self, nx=nx, ny=ny, nz=nz,
                       n_sources=max(min_sources, int(round(self.n_sources * k))))


# The workloads: a tiny cube, one GPU's 16 GiB brick, 64 uneven items, the
# resident set of a server, and a precision stress cube at a large offset.
WORKLOADS = {
    "tiny": Recipe(64, 64, 128, n_sources=20, amp_dist="uniform", amp_lo=5, amp_hi=50,
                   p_voxel_nan=0.01),
    "brick16g": Recipe(2048, 2048, 1024, n_sources=10_000, amp_dist="loguniform",
                       amp_lo=3, amp_hi=1000, p_pixel_nan=0.005, chan_nan_frac=0.005,
                       chan_nan_ranges=3),
    "stress128g": Recipe(4096, 4096, 2048, n_sources=100_000, amp_dist="loguniform",
                         amp_lo=1e-2, amp_hi=1e3, offset=1e4, noise_sigma=1e-3,
                         p_pixel_nan=0.01, chan_nan_frac=0.01, chan_nan_ranges=3),
}
HIST_BINS = {"tiny": 256, "brick16g": 1024, "batch64": 512, "stress128g": 4096}


def batch_item_recipes(seed: int = BASE_SEED + 2, n_items: int = 64):
    """64 uneven items: nx, ny log-uniform in [32, 512], nz log-uniform in
    [32, 256]; each item noise + 20 sources with peak U[5, 50] and 0.5 % NaN."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_items):
        nx, ny = (int(math.exp(rng.uniform(math.log(32), math.log(512)))) for _ in range(2))
        nz = int(math.exp(rng.uniform(math.log(32), math.log(256))))
        out.append(Recipe(nx, ny, nz, n_sources=20, amp_dist="uniform", amp_lo=5,
                          amp_hi=50, p_voxel_nan=0.005))
    return out


SERVE_SHAPES = [  # (nx, ny, nz): twelve resident cubes, about 201 GiB together
    (4096, 4096, 1024), (4096, 4096, 512), (4096, 2048, 1024), (2048, 2048, 1024),
    (2048, 2048, 1024), (4096, 2048, 512), (2048, 2048, 512), (2048, 2048, 512),
    (2048, 1024, 512), (1024, 1024, 1024), (1024, 1024, 256), (512, 512, 256),
]


def serve_recipes(scale_div: int = 1):
    """The resident set, built like the 16 GiB brick (10^4 sources per 2^32
    voxels).  ``scale_div`` shrinks every axis (for small test runs)."""
    base = WORKLOADS["brick16g"]
    return [base.scaled(max(8, a // scale_div), max(8, b // scale_div), max(8, c // scale_div))
            for a, b, c in SERVE_SHAPES]


@dataclass
class Drawn:
    """Host-side random draws of a recipe: sources, tile lists, channel ranges."""
    src: np.ndarray            # float64 [n_sources, 4]: cx, cy, cz, amp
    tile_start: np.ndarray     # int32 [n_tiles + 1]
    src_idx: np.ndarray        # int32
    tiles: tuple
    chan_ranges: list = field(default_factory=list)


def draw(r: Recipe, seed: int) -> Drawn:
    rng = np.random.default_rng([seed, 0x5EED])
    ns = r.n_sources
    cx = rng.uniform(0, r.nx, ns)
    cy = rng.uniform(0, r.ny, ns)
    cz = rng.uniform(0, r.nz, ns)
    if r.amp_dist == "uniform":
        amp = rng.uniform(r.amp_lo, r.amp_hi, ns)
    elif r.amp_dist == "loguniform":
        amp = np.exp(rng.uniform(math.log(r.amp_lo), math.log(r.amp_hi), ns))
    else:
        raise ValueError(r.amp_dist)
    src = np.stack([cx, cy, cz, amp], axis=1).astype(np.float64) if ns else np.zeros((0, 4))

    tx, ty, tz = (-(-r.nx // TILE), -(-r.ny // TILE), -(-r.nz // TILE))
    pairs_t, pairs_s = [], []
    rad = r.radius
    for s in range(ns):
        lo = [max(0, math.ceil(c - q)) for c, q in zip(src[s, :3], rad)]
        hi = [min(n - 1, math.floor(c + q)) for c, q, n in zip(src[s, :3], rad, (r.nx, r.ny, r.nz))]
        if any(a > b for a, b in zip(lo, hi)):
            continue
        for kz in range(lo[2] // TILE, hi[2] // TILE + 1):
            for ky in range(lo[1] // TILE, hi[1] // TILE + 1):
                for kx in range(lo[0] // TILE, hi[0] // TILE + 1):
                    pairs_t.append(kx + tx * (ky + ty * kz))
                    pairs_s.append(s)
    pairs_t = np.asarray(pairs_t, dtype=np.int64)
    pairs_s = np.asarray(pairs_s, dtype=np.int64)
    order = np.lexsort((pairs_s, pairs_t))          # by tile, then source index
    n_tiles = tx * ty * tz
    counts = np.bincount(pairs_t, minlength=n_tiles) if len(pairs_t) else np.zeros(n_tiles, np.int64)
    tile_start = np.zeros(n_tiles + 1, dtype=np.int32)
    tile_start[1:] = np.cumsum(counts)
    src_idx = pairs_s[order].astype(np.int32)

    chan = []
    if r.chan_nan_ranges and r.chan_nan_frac > 0:
        total = max(1, int(round(r.chan_nan_frac * r.nz)))
        k = min(r.chan_nan_ranges, total)
        sizes = np.full(k, total // k)
        sizes[: total % k] += 1
        # Non-overlapping ranges at random positions (gaps drawn, then placed).
        free = r.nz - total
        cuts = np.sort(rng.integers(0, free + 1, k))
        pos = 0
        for i in range(k):
            start = int(cuts[i]) + pos
            chan.append((start, start + int(sizes[i])))
            pos += int(sizes[i])
    return Drawn(src, tile_start, src_idx if len(src_idx) else np.zeros(1, np.int32),
                 (tx, ty, tz), chan)


# ---------------------------------------------------------------- numpy version
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _hash3(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        k = np.uint64(seed) ^ (np.uint64(stream) * np.uint64(0xD1B54A32D192ED03))
        key = _splitmix64(np.asarray([k], dtype=np.uint64))[0]
        return _splitmix64(key + idx.astype(np.uint64))


def _unit_open(h: np.ndarray) -> np.ndarray:
    return ((h >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def make_numpy(r: Recipe, seed: int) -> np.ndarray:
    """The recipe as a dense float32 array indexed [z, y, x] (small cubes only)."""
    d = draw(r, seed)
    v = np.arange(r.n, dtype=np.uint64)
    u1 = _unit_open(_hash3(seed, 1, v))
    u2 = _unit_open(_hash3(seed, 2, v))
    val = r.offset + r.noise_sigma * np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
    val = val.reshape(r.nz, r.ny, r.nx)
    sg = r.sigma
    for s in range(r.n_sources):
        cx, cy, cz, a = d.src[s]
        lo = [max(0, math.ceil(c - q)) for c, q in zip((cx, cy, cz), r.radius)]
        hi = [min(n - 1, math.floor(c + q)) for c, q, n in zip((cx, cy, cz), r.radius, (r.nx, r.ny, r.nz))]
        if any(p > q for p, q in zip(lo, hi)):
            continue
        xs = np.arange(lo[0], hi[0] + 1) - cx
        ys = np.arange(lo[1], hi[1] + 1) - cy
        zs = np.arange(lo[2], hi[2] + 1) - cz
        q = (zs[:, None, None] ** 2 / (sg[2] * sg[2]) + ys[None, :, None] ** 2 / (sg[1] * sg[1])
             + xs[None, None, :] ** 2 / (sg[0] * sg[0]))
        val[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += a * np.exp(-0.5 * q)
    out = val.astype(np.float32)
    blank = np.zeros(r.n, dtype=bool)
    if r.p_voxel_nan > 0:
        blank |= _unit_open(_hash3(seed, 3, v)) < r.p_voxel_nan
    blank = blank.reshape(r.nz, r.ny, r.nx)
    if r.p_pixel_nan > 0:
        pix = np.arange(r.nx * r.ny, dtype=np.uint64)
        blank |= (_unit_open(_hash3(seed, 4, pix)) < r.p_pixel_nan).reshape(1, r.ny, r.nx)
    for a, b in d.chan_ranges:
        blank[a:b] = True
    out[blank] = np.float32(np.nan)
    return out


# ---------------------------------------------------------------- HIP version
class _RecipeC(C.Structure):
    _fields_ = [("seed", C.c_uint64),
                ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("sy", C.c_int64), ("sz", C.c_int64),
                ("offset", C.c_double), ("noise_sigma", C.c_double),
                ("sig_x", C.c_double), ("sig_y", C.c_double), ("sig_z", C.c_double),
                ("rad_x", C.c_int32), ("rad_y", C.c_int32), ("rad_z", C.c_int32),
                ("n_chan_ranges", C.c_int32),
                ("p_voxel_nan", C.c_double), ("p_pixel_nan", C.c_double),
                ("chan_lo", C.c_int32 * 8), ("chan_hi", C.c_int32 * 8),
                ("src", C.c_void_p), ("n_sources", C.c_int64),
                ("tile_start", C.c_void_p), ("src_idx", C.c_void_p),
                ("tiles_x", C.c_int64), ("tiles_y", C.c_int64), ("tiles_z", C.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        lib.synth_fill_box.argtypes = [C.POINTER(_RecipeC), C.c_void_p, C.c_void_p]
        lib.synth_fill_box.restype = C.c_int
        lib.synth_recipe_size.restype = C.c_int
        if lib.synth_recipe_size() != C.sizeof(_RecipeC):
            raise RuntimeError("synth recipe layout mismatch")
        _lib = lib
    return _lib


def fill_device(r: Recipe, seed: int, ptr: int, sy: int | None = None,
                sz: int | None = None, stream: int = 0, device=None) -> None:
    """Write the recipe into the float32 box at device address ``ptr``.

    Pitches default to a dense cube.  Synchronous: returns after the fill.
    """
    import torch
    lib = _load()
    d = draw(r, seed)
    if len(d.chan_ranges) > 8:
        raise ValueError("at most 8 blanked channel ranges")
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    src_t = torch.from_numpy(np.ascontiguousarray(d.src if len(d.src) else np.zeros((1, 4)))).to(dev)
    ts_t = torch.from_numpy(d.tile_start).to(dev)
    si_t = torch.from_numpy(np.ascontiguousarray(d.src_idx)).to(dev)
    n_tiles = d.tiles[0] * d.tiles[1] * d.tiles[2]
    assert len(d.tile_start) == n_tiles + 1
    assert d.tile_start[-1] <= len(d.src_idx)
    assert r.n_sources == 0 or int(d.src_idx.max()) < len(d.src)
    rc = _RecipeC()
    rc.seed = seed
    rc.nx, rc.ny, rc.nz = r.nx, r.ny, r.nz
    rc.sy = r.nx if sy is None else sy
    rc.sz = rc.sy * r.ny if sz is None else sz
    rc.offset, rc.noise_sigma = r.offset, r.noise_sigma
    rc.sig_x, rc.sig_y, rc.sig_z = r.sigma
    rc.rad_x, rc.rad_y, rc.rad_z = r.radius
    rc.n_chan_ranges = len(d.chan_ranges)
    for i, (a, b) in enumerate(d.chan_ranges):
        rc.chan_lo[i], rc.chan_hi[i] = a, b
    rc.p_voxel_nan, rc.p_pixel_nan = r.p_voxel_nan, r.p_pixel_nan
    rc.src, rc.n_sources = src_t.data_ptr(), r.n_sources
    rc.tile_start, rc.src_idx = ts_t.data_ptr(), si_t.data_ptr()
    rc.tiles_x, rc.tiles_y, rc.tiles_z = d.tiles
    err = lib.synth_fill_box(C.byref(rc), C.c_void_p(ptr), C.c_void_p(stream))
    if err != 0:
        raise RuntimeError(f"synth_fill_box failed: HIP error {err}")
    torch.cuda.synchronize(dev)
    del src_t, ts_t, si_t


def cube_tensor(r: Recipe, seed: int, device="cuda"):
    """A new dense device tensor [nz, ny, nx] holding the recipe."""
    import torch
    t = torch.empty((r.nz, r.ny, r.nx), dtype=torch.float32, device=device)
    fill_device(r, seed, t.data_ptr(), device=t.device)
    return t
