"""Query streams for the serving measurement (synthetic, seeded).

A query stream over resident cubes: Poisson arrivals; each query picks a
cube uniformly; 40 % full-cube statistics, 30 % sub-region statistics, 30 %
fused statistics + histogram (half full cube, half sub-region) with nbins in
{64, 256, 1024, 4096} and a given range (half the cube's [min, max], half
[mean - 2 std, mean + 2 std]).  A sub-region covers a volume fraction f drawn
log-uniform in [0.01, 0.5], split over the axes as f^w with w ~ Dirichlet(2,
2, 2), at a random origin.  This module only draws query parameters; it
computes nothing of the statistics.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class QuerySpec:
    t_arrival: float      # seconds from the start of the stream
    cube: int
    box: tuple            # (z0, z1, y0, y1, x0, x1)
    kind: int             # CUBE_Q_STATS or CUBE_Q_FUSED
    nbins: int
    lo: float
    hi: float

    @property
    def voxels(self) -> int:
        z0, z1, y0, y1, x0, x1 = self.box
        return (z1 - z0) * (y1 - y0) * (x1 - x0)


def _sub_box(rng, shape):
    nz, ny, nx = shape
    f = math.exp(rng.uniform(math.log(0.01), math.log(0.5)))
    w = rng.dirichlet([2.0, 2.0, 2.0])
    ext = []
    for n, wi in zip((nz, ny, nx), w):
        e = max(1, min(n, int(round(n * f ** wi))))
        o = int(rng.integers(0, n - e + 1))
        ext += [o, o + e]
    return tuple(ext)


def query_stream(shapes, ranges, n: int, qps: float, seed: int, stats_kind: int,
                 fused_kind: int):
    """n queries at mean rate qps.  shapes: [(nz, ny, nx)] per cube; ranges:
    per cube ((min, max), (mean - 2 std, mean + 2 std))."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0 / qps)
        c = int(rng.integers(len(shapes)))
        nz, ny, nx = shapes[c]
        u = rng.random()
        if u < 0.4:
            out.append(QuerySpec(t, c, (0, nz, 0, ny, 0, nx), stats_kind, 0, 0.0, 0.0))
        elif u < 0.7:
            out.append(QuerySpec(t, c, _sub_box(rng, shapes[c]), stats_kind, 0, 0.0, 0.0))
        else:
            box = (0, nz, 0, ny, 0, nx) if rng.random() < 0.5 else _sub_box(rng, shapes[c])
            nb = int(rng.choice([64, 256, 1024, 4096]))
            lo, hi = ranges[c][int(rng.integers(2))]
            out.append(QuerySpec(t, c, box, fused_kind, nb, float(lo), float(hi)))
    return out
