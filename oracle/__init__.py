"""CPU oracle for the cube statistics + histogram pass (ctypes wrapper).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never loads it, and it shares no code with the GPU library.

The arithmetic lives in ``cubeoracle.c`` (plain single-threaded C in FP64; see
its header for the definitions, which follow the tasks named in the paper's
Abstract and Section 3).  This module only marshals numpy arrays into it.

Every function takes a numpy ``float32`` array: either a 3-D array indexed
``[z, y, x]`` (the channel axis z slowest, x fastest), any strided view with a
unit x-stride, or a 1-D array (treated as nx = len, ny = nz = 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cubeoracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORACLE_ABI = 2   # layout of the sweep records; equals ORACLE_ABI in cubeoracle.c

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fno-unsafe-math-optimizations", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build() -> str:
    """Compile the oracle with gcc.  Always recompiles."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Sweep1(C.Structure):
    _fields_ = [("n_total", C.c_uint64), ("n_valid", C.c_uint64), ("n_nan", C.c_uint64),
                ("min", C.c_float), ("max", C.c_float),
                ("sum", C.c_double), ("sum_c", C.c_double),
                ("sabs", C.c_double), ("sabs_c", C.c_double),
                ("n_pinf", C.c_uint64), ("n_ninf", C.c_uint64)]


class _Sweep2(C.Structure):
    _fields_ = [("n", C.c_uint64), ("dev", C.c_double), ("dev_c", C.c_double),
                ("sq", C.c_double), ("sq_c", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("n_total", C.c_uint64), ("n_valid", C.c_uint64), ("n_nan", C.c_uint64),
                ("min", C.c_float), ("max", C.c_float),
                ("mean", C.c_double), ("m2", C.c_double), ("std", C.c_double),
                ("mean_abs", C.c_double)]


@dataclass
class Stats:
    n_total: int
    n_valid: int
    n_nan: int
    min: float
    max: float
    mean: float
    m2: float
    std: float
    mean_abs: float


class Oracle:
    """The oracle library loaded from one shared object (by default the one
    ``build()`` writes; the mutation tests load deliberately broken copies)."""

    def __init__(self, path: str | None = None):
        if path is None:
            path = _LIB
            if not os.path.exists(path):
                build()
        lib = C.CDLL(path)
        i64, f32, f64 = C.c_int64, C.c_float, C.c_double
        P = C.c_void_p
        lib.oracle_abi_version.restype = C.c_int
        if lib.oracle_abi_version() != ORACLE_ABI:
            raise RuntimeError(f"{path}: oracle ABI {lib.oracle_abi_version()}, "
                               f"expected {ORACLE_ABI}: rebuild it (oracle.build())")
        lib.oracle_sweep1_init.argtypes = [C.POINTER(_Sweep1)]
        lib.oracle_sweep1.argtypes = [C.POINTER(_Sweep1), P, i64, i64, i64, i64, i64]
        lib.oracle_sweep1.restype = C.c_int
        lib.oracle_sweep1_mean.argtypes = [C.POINTER(_Sweep1)]
        lib.oracle_sweep1_mean.restype = f64
        lib.oracle_sweep2_init.argtypes = [C.POINTER(_Sweep2)]
        lib.oracle_sweep2.argtypes = [C.POINTER(_Sweep2), P, i64, i64, i64, i64, i64, f64]
        lib.oracle_sweep2.restype = C.c_int
        lib.oracle_finish.argtypes = [C.POINTER(_Sweep1), C.POINTER(_Sweep2),
                                      C.POINTER(_Stats)]
        lib.oracle_sweep1_add.argtypes = [C.POINTER(_Sweep1), C.POINTER(_Sweep1)]
        lib.oracle_sweep2_add.argtypes = [C.POINTER(_Sweep2), C.POINTER(_Sweep2)]
        lib.oracle_stats.argtypes = [P, i64, i64, i64, i64, i64, C.POINTER(_Stats)]
        lib.oracle_stats.restype = C.c_int
        lib.oracle_hist_scale.argtypes = [f32, f32, C.c_int32, C.POINTER(f32)]
        lib.oracle_hist_scale.restype = C.c_int
        lib.oracle_hist.argtypes = [P, i64, i64, i64, i64, i64, f32, f32, C.c_int32, P]
        lib.oracle_hist.restype = C.c_int
        lib.oracle_hist_accumulate.argtypes = lib.oracle_hist.argtypes
        lib.oracle_hist_accumulate.restype = C.c_int
        lib.oracle_select.argtypes = [P, i64, i64, i64, i64, i64, C.c_uint64, C.POINTER(f32)]
        lib.oracle_select.restype = C.c_int
        lib.oracle_median.argtypes = [P, i64, i64, i64, i64, i64, C.POINTER(f64),
                                      C.POINTER(C.c_uint64)]
        lib.oracle_median.restype = C.c_int
        lib.oracle_quantiles.argtypes = [P, i64, i64, i64, i64, i64, P, C.c_int32, P,
                                         C.POINTER(C.c_uint64)]
        lib.oracle_quantiles.restype = C.c_int
        lib.oracle_project.argtypes = [P, i64, i64, i64, i64, i64, P, P, P]
        lib.oracle_project.restype = C.c_int
        self.lib = lib
        self.path = path

    def stats(self, a: np.ndarray) -> Stats:
        """All statistics of one box (two sweeps)."""
        ptr, nx, ny, nz, sy, sz = box_of(a)
        out = _Stats()
        if self.lib.oracle_stats(ptr, nx, ny, nz, sy, sz, C.byref(out)) != 0:
            raise ValueError("invalid box")
        return Stats(*(getattr(out, f[0]) for f in _Stats._fields_))

    def stats_pieces(self, pieces) -> Stats:
        """Statistics of a cube given as a re-iterable sequence of pieces.

        ``pieces`` is a callable returning an iterator of float32 arrays; it is
        called twice (one call per sweep), so a cube larger than host memory
        can be streamed from the device piece by piece.
        """
        lib = self.lib
        s1, s2, out = _Sweep1(), _Sweep2(), _Stats()
        lib.oracle_sweep1_init(C.byref(s1))
        for a in pieces():
            if lib.oracle_sweep1(C.byref(s1), *box_of(a)) != 0:
                raise ValueError("invalid box")
        mean = lib.oracle_sweep1_mean(C.byref(s1))
        lib.oracle_sweep2_init(C.byref(s2))
        for a in pieces():
            if lib.oracle_sweep2(C.byref(s2), *box_of(a), mean) != 0:
                raise ValueError("invalid box")
        lib.oracle_finish(C.byref(s1), C.byref(s2), C.byref(out))
        return Stats(*(getattr(out, f[0]) for f in _Stats._fields_))

    def stats_slabs(self, slabs, threads: int) -> Stats:
        """Statistics of a cube given as consecutive slabs, swept side by side.

        ``slabs`` is a list of callables, one per slab in cube order, each
        returning an iterator of float32 arrays (the slab's pieces, as for
        ``stats_pieces``); each is called twice.  Every slab is swept into a
        record of its own on one of ``threads`` host threads (the C sweeps
        release the GIL), and the records are added in slab order, so the
        result is that of one sweep over the whole cube up to the rounding
        of the compensated sums.
        """
        from concurrent.futures import ThreadPoolExecutor
        lib = self.lib

        def sweep1(pieces):
            s = _Sweep1()
            lib.oracle_sweep1_init(C.byref(s))
            for a in pieces():
                if lib.oracle_sweep1(C.byref(s), *box_of(a)) != 0:
                    raise ValueError("invalid box")
            return s

        with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            r1 = list(ex.map(sweep1, slabs))
            s1 = _Sweep1()
            lib.oracle_sweep1_init(C.byref(s1))
            for r in r1:
                lib.oracle_sweep1_add(C.byref(s1), C.byref(r))
            mean = lib.oracle_sweep1_mean(C.byref(s1))

            def sweep2(pieces):
                s = _Sweep2()
                lib.oracle_sweep2_init(C.byref(s))
                for a in pieces():
                    if lib.oracle_sweep2(C.byref(s), *box_of(a), mean) != 0:
                        raise ValueError("invalid box")
                return s

            r2 = list(ex.map(sweep2, slabs))
        s2, out = _Sweep2(), _Stats()
        lib.oracle_sweep2_init(C.byref(s2))
        for r in r2:
            lib.oracle_sweep2_add(C.byref(s2), C.byref(r))
        lib.oracle_finish(C.byref(s1), C.byref(s2), C.byref(out))
        return Stats(*(getattr(out, f[0]) for f in _Stats._fields_))

    def select(self, a: np.ndarray, k: int) -> float:
        """The valid voxel of rank k (0-based; -0 orders before +0)."""
        v = C.c_float()
        rc = self.lib.oracle_select(*box_of(a), k, C.byref(v))
        if rc != 0:
            raise ValueError("invalid box or rank")
        return v.value

    def median(self, a: np.ndarray) -> float:
        """Median of the valid voxels (mean of the two middle ones if even)."""
        m, n = C.c_double(), C.c_uint64()
        if self.lib.oracle_median(*box_of(a), C.byref(m), C.byref(n)) != 0:
            raise ValueError("no valid voxel or invalid box")
        return m.value

    def quantiles(self, a: np.ndarray, q) -> np.ndarray:
        """Quantiles (linear interpolation between the valid voxels around
        rank q * (n_valid - 1)) at the levels q, as float64."""
        qa = np.ascontiguousarray(np.atleast_1d(np.asarray(q, dtype=np.float64)))
        out = np.empty(qa.size, dtype=np.float64)
        n = C.c_uint64()
        rc = self.lib.oracle_quantiles(*box_of(a), qa.ctypes.data, qa.size, out.ctypes.data,
                                       C.byref(n))
        if rc != 0:
            raise ValueError("invalid box, level outside [0, 1], or no valid voxel")
        return out

    def project(self, a: np.ndarray):
        """(mip float32 [ny, nx], mom0 float64 [ny, nx], nvalid uint32 [ny, nx])
        of a [z, y, x] array: projections along the channel axis z."""
        ptr, nx, ny, nz, sy, sz = box_of(a)
        mip = np.empty((ny, nx), np.float32)
        mom0 = np.empty((ny, nx), np.float64)
        nv = np.empty((ny, nx), np.uint32)
        if self.lib.oracle_project(ptr, nx, ny, nz, sy, sz, mip.ctypes.data, mom0.ctypes.data,
                                   nv.ctypes.data) != 0:
            raise ValueError("invalid box")
        return mip, mom0, nv

    def hist_scale(self, lo: float, hi: float, nbins: int) -> float:
        """The FP32 scale nbins / (hi - lo); ValueError on an invalid range."""
        s = C.c_float()
        if self.lib.oracle_hist_scale(C.c_float(lo), C.c_float(hi), nbins,
                                      C.byref(s)) != 0:
            raise ValueError("invalid histogram range")
        return s.value

    def hist(self, a: np.ndarray, lo: float, hi: float, nbins: int) -> np.ndarray:
        """uint64 counts[nbins + 3]: the bins, then below, above and NaN."""
        if nbins < 1 or nbins > 65536:
            raise ValueError("nbins out of range")
        counts = np.zeros(nbins + 3, dtype=np.uint64)
        rc = self.lib.oracle_hist(*box_of(a), C.c_float(lo), C.c_float(hi), nbins,
                                  counts.ctypes.data)
        if rc != 0:
            raise ValueError("invalid box or histogram range")
        return counts

    def hist_pieces(self, pieces, lo: float, hi: float, nbins: int) -> np.ndarray:
        """Histogram of a cube given as pieces (see ``stats_pieces``)."""
        if nbins < 1 or nbins > 65536:
            raise ValueError("nbins out of range")
        counts = np.zeros(nbins + 3, dtype=np.uint64)
        for a in pieces():
            rc = self.lib.oracle_hist_accumulate(*box_of(a), C.c_float(lo),
                                                 C.c_float(hi), nbins,
                                                 counts.ctypes.data)
            if rc != 0:
                raise ValueError("invalid box or histogram range")
        return counts


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def stats(a):
    return default().stats(a)


def stats_pieces(pieces):
    return default().stats_pieces(pieces)


def stats_slabs(slabs, threads):
    return default().stats_slabs(slabs, threads)


def hist_scale(lo, hi, nbins):
    return default().hist_scale(lo, hi, nbins)


def hist(a, lo, hi, nbins):
    return default().hist(a, lo, hi, nbins)


def hist_pieces(pieces, lo, hi, nbins):
    return default().hist_pieces(pieces, lo, hi, nbins)


def select(a, k):
    return default().select(a, k)


def median(a):
    return default().median(a)


def quantiles(a, q):
    return default().quantiles(a, q)


def project(a):
    return default().project(a)


def box_of(a: np.ndarray):
    """(pointer, nx, ny, nz, sy, sz) of a float32 array with unit x-stride."""
    if a.dtype != np.float32:
        raise TypeError("oracle takes float32 arrays")
    if a.ndim == 1:
        a3 = a.reshape(1, 1, -1) if a.strides[0] == 4 else None
        if a3 is None:
            raise ValueError("1-D input must be contiguous")
        a = a3
    if a.ndim != 3:
        raise ValueError("oracle takes 1-D or 3-D [z, y, x] arrays")
    nz, ny, nx = a.shape
    sz, sy, sx = (s // 4 for s in a.strides)
    if nx > 1 and sx != 1:
        raise ValueError("x stride must be 1")
    if any(s % 4 for s in a.strides):
        raise ValueError("strides must be whole floats")
    ptr = a.__array_interface__["data"][0]
    return ptr, nx, ny, nz, sy, sz

