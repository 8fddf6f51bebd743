"""Streaming a device cube to the oracle, slab by slab, on host threads.

A cube too large for one host copy (the 128 GiB stress cube) is cut into
consecutive channel slabs; each slab is copied to the host a chunk of planes
at a time and swept by the oracle on a thread of its own
(``oracle.stats_slabs``), and the slab records are added in slab order.  The
slab layout is fixed by ``SLAB_PLANES`` alone, so the result does not depend
on the number of threads.
"""
from __future__ import annotations

import os

SLAB_PLANES = 128     # planes per slab (the unit of work of one thread)
CHUNK_PLANES = 16     # planes per host copy within a slab


def host_threads(cap: int = 16) -> int:
    """Host threads for the oracle sweeps: the CPUs this process may use,
    at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def device_slabs(t, slab_planes: int = SLAB_PLANES, chunk_planes: int = CHUNK_PLANES):
    """One callable per slab of the [z, y, x] device tensor `t`; each returns
    an iterator of host float32 arrays (the slab's planes, chunk by chunk)."""
    nz = t.shape[0]

    def slab(z0: int, z1: int):
        def pieces():
            for c0 in range(z0, z1, chunk_planes):
                yield t[c0:min(z1, c0 + chunk_planes)].cpu().numpy()
        return pieces

    return [slab(z0, min(nz, z0 + slab_planes)) for z0 in range(0, nz, slab_planes)]


def oracle_stats_of_device(oracle_mod, t, threads: int | None = None):
    """The oracle's statistics of the whole device tensor `t`."""
    return oracle_mod.stats_slabs(device_slabs(t), threads or host_threads())
