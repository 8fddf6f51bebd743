"""MI355X cube statistics + histogram engine: Python binding of libcubestats.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libcubestats.so`` (see ``include/cubestats.h`` for the contract).
The binding fails loudly when the library is missing or no GPU is present;
there is no CPU fallback.

Two layers:
  * the C entry points under the same names (``cube_stats``, ``cube_hist``,
    ``cube_stats_hist``, ``cube_stats_hist_minmax`` and the ``*_async``
    forms), taking raw device addresses and integers;
  * tensor helpers (``stats``, ``hist``, ``stats_hist``, ``stats_hist_minmax``)
    that take a float32 torch tensor on the GPU -- 1-D, or 3-D indexed
    [z, y, x] with unit x-stride -- and marshal its address and pitches.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcubestats.so")

CUBE_OK, CUBE_EINVAL, CUBE_ENOMEM, CUBE_EDEVICE, CUBE_EBUSY = 0, -1, -2, -3, -4
CUBE_MAX_BINS = 65536
CUBE_NO_VALID, CUBE_HIST_BAD_RANGE = 1, 2
CUBE_ACCUM_FP64MERGE, CUBE_ACCUM_KAHAN32, CUBE_ACCUM_NAIVE32 = 0, 1, 2
CUBE_HIST_AUTO, CUBE_HIST_PLAIN, CUBE_HIST_HOT = 0, 1, 2
CUBE_PARTITION_AUTO, CUBE_PARTITION_STATIC = 0, 1
CUBE_CHUNK_LOG2_MIN, CUBE_CHUNK_LOG2_MAX = 12, 26


class CubeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cubestats error {code}: {msg}")
        self.code = code


class cube_stats_t(C.Structure):
    _fields_ = [("n_total", C.c_uint64), ("n_valid", C.c_uint64), ("n_nan", C.c_uint64),
                ("min", C.c_float), ("max", C.c_float),
                ("mean", C.c_double), ("m2", C.c_double), ("std", C.c_double),
                ("flags", C.c_uint32), ("reserved", C.c_uint32)]


assert C.sizeof(cube_stats_t) == 64

CUBE_Q_STATS, CUBE_Q_HIST, CUBE_Q_FUSED, CUBE_Q_MINMAX = 0, 1, 2, 3
CUBE_ORDER_LARGEST_FIRST, CUBE_ORDER_SMALLEST_FIRST = 0, 1


class cube_query_t(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("dims", C.c_int64 * 5), ("kind", C.c_int32),
                ("nbins", C.c_int32), ("lo", C.c_float), ("hi", C.c_float),
                ("out", C.c_void_p), ("counts", C.c_void_p)]


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
    flags: int

    @classmethod
    def from_c(cls, s: cube_stats_t) -> "Stats":
        return cls(s.n_total, s.n_valid, s.n_nan, s.min, s.max, s.mean, s.m2, s.std, s.flags)

    @classmethod
    def from_bytes(cls, b: bytes) -> "Stats":
        return cls.from_c(cube_stats_t.from_buffer_copy(b))


_lib = None


def load() -> C.CDLL:
    """Load libcubestats.so (built in-tree by ``build.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1111_6661_amd/build.py "
                           "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    I64P = C.POINTER(C.c_int64)
    lib.cube_abi_version.restype = C.c_int
    lib.cube_last_error.restype = C.c_char_p
    lib.cube_stats.argtypes = [P, i64, i64, i64, I64P, P]
    lib.cube_hist.argtypes = [P, I64P, f32, f32, i32, P]
    lib.cube_stats_hist.argtypes = [P, I64P, f32, f32, i32, P, P]
    lib.cube_stats_hist_minmax.argtypes = [P, I64P, i32, P, P]
    lib.cube_stats_async.argtypes = [P, I64P, P, P]
    lib.cube_hist_async.argtypes = [P, I64P, f32, f32, i32, P, P]
    lib.cube_stats_hist_async.argtypes = [P, I64P, f32, f32, i32, P, P, P]
    lib.cube_stats_hist_minmax_async.argtypes = [P, I64P, i32, P, P, P]
    lib.cube_stats_hist_noalloc.argtypes = [P, I64P, f32, f32, i32, P, P, P]
    lib.cube_set_accum_mode.argtypes = [i32]
    lib.cube_set_launch.argtypes = [i32, i32, i32, i32]
    lib.cube_set_hist_mode.argtypes = [i32]
    lib.cube_set_partition.argtypes = [i32]
    lib.cube_describe_plan.argtypes = [P, I64P, i32, i32, C.c_char_p, C.c_size_t]
    lib.cube_shutdown.restype = None
    lib.cube_release_stream.argtypes = [P]
    lib.cube_release_stream.restype = None
    lib.cube_batch_create.argtypes = [C.POINTER(C.c_void_p)]
    lib.cube_batch_destroy.argtypes = [P]
    lib.cube_batch_destroy.restype = None
    lib.cube_batch_set_tile.argtypes = [P, i64, i32]
    lib.cube_batch_enqueue.argtypes = [P, C.POINTER(cube_query_t), i32, P]
    lib.cube_batch_relaunch.argtypes = [P, P]
    lib.cube_batch_set_order.argtypes = [P, i32]
    lib.cube_batch_query_done.argtypes = [P, i32]
    lib.cube_batch_graph_launch.argtypes = [P, P]
    lib.cube_batch_check.argtypes = [P]
    lib.cube_batch_run.argtypes = [C.POINTER(cube_query_t), i32]
    lib.cube_server_create.argtypes = [i32, i32, i32, i64, i64, C.POINTER(C.c_void_p)]
    lib.cube_server_submit.argtypes = [P, C.POINTER(cube_query_t), C.POINTER(C.c_uint64)]
    lib.cube_server_wait.argtypes = [P, C.c_uint64, C.c_double, C.POINTER(C.c_double)]
    lib.cube_server_latency.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_uint64), i32]
    lib.cube_project.argtypes = [P, I64P, P, P, P, P]
    lib.cube_project.restype = C.c_int
    lib.cube_read_probe.argtypes = [P, I64P, i32, P, P]
    lib.cube_read_probe.restype = C.c_int
    lib.cube_host_query.argtypes = [C.POINTER(cube_query_t), i64]
    lib.cube_host_query.restype = C.c_int
    lib.cube_select.argtypes = [P, I64P, C.c_uint64, C.POINTER(C.c_float)]
    lib.cube_select.restype = C.c_int
    lib.cube_median.argtypes = [P, I64P, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    lib.cube_median.restype = C.c_int
    lib.cube_quantiles.argtypes = [P, I64P, P, i32, P, C.POINTER(C.c_uint64)]
    lib.cube_quantiles.restype = C.c_int
    lib.cube_last_quantile_reads.argtypes = []
    lib.cube_last_quantile_reads.restype = C.c_int
    lib.cube_autotune.argtypes = [P, I64P, i32, f32, f32, i32, i32, C.c_char_p, C.c_size_t]
    lib.cube_autotune.restype = C.c_int
    lib.cube_autotune_batch.argtypes = [C.POINTER(cube_query_t), i32, i32, C.c_char_p, C.c_size_t]
    lib.cube_autotune_batch.restype = C.c_int
    lib.cube_tune_save.argtypes = [C.c_char_p]
    lib.cube_tune_save.restype = C.c_int
    lib.cube_tune_load.argtypes = [C.c_char_p]
    lib.cube_tune_load.restype = C.c_int
    lib.cube_tune_clear.restype = None
    lib.cube_server_destroy.argtypes = [P]
    lib.cube_server_destroy.restype = None
    for name in ("cube_server_create", "cube_server_submit", "cube_server_wait",
                 "cube_server_latency"):
        getattr(lib, name).restype = C.c_int
    for name in ("cube_batch_create", "cube_batch_set_tile", "cube_batch_enqueue",
                 "cube_batch_set_order", "cube_batch_query_done",
                 "cube_batch_relaunch", "cube_batch_graph_launch", "cube_batch_check",
                 "cube_batch_run"):
        getattr(lib, name).restype = C.c_int
    for name in ("cube_stats", "cube_hist", "cube_stats_hist", "cube_stats_hist_minmax",
                 "cube_stats_async", "cube_hist_async", "cube_stats_hist_async",
                 "cube_stats_hist_minmax_async", "cube_stats_hist_noalloc",
                 "cube_set_accum_mode", "cube_set_launch", "cube_set_hist_mode",
                 "cube_set_partition", "cube_describe_plan"):
        getattr(lib, name).restype = C.c_int
    if lib.cube_abi_version() != 1:
        raise RuntimeError("libcubestats ABI version mismatch")
    _lib = lib
    return lib


def last_error() -> str:
    return load().cube_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise CubeError(rc, last_error())
    return rc


def _dims(dims) -> C.Array:
    d = list(dims) + [0] * (5 - len(dims))
    return (C.c_int64 * 5)(*d)


# ------------------------------------------------------------ C entry points
def cube_stats(ptr: int, nx: int, ny: int, nz: int, stride=None) -> Stats:
    out = cube_stats_t()
    st = (C.c_int64 * 2)(*stride) if stride is not None else None
    _check(load().cube_stats(C.c_void_p(ptr), nx, ny, nz, st, C.byref(out)))
    return Stats.from_c(out)


def cube_hist(ptr: int, dims, lo: float, hi: float, nbins: int) -> np.ndarray:
    counts = np.zeros(max(nbins, 0) + 3, dtype=np.uint64)
    _check(load().cube_hist(C.c_void_p(ptr), _dims(dims), lo, hi, nbins, counts.ctypes.data))
    return counts


def cube_stats_hist(ptr: int, dims, lo: float, hi: float, nbins: int):
    out = cube_stats_t()
    counts = np.zeros(max(nbins, 0) + 3, dtype=np.uint64)
    _check(load().cube_stats_hist(C.c_void_p(ptr), _dims(dims), lo, hi, nbins, C.byref(out),
                                  counts.ctypes.data))
    return Stats.from_c(out), counts


def cube_stats_hist_minmax(ptr: int, dims, nbins: int):
    out = cube_stats_t()
    counts = np.zeros(max(nbins, 0) + 3, dtype=np.uint64)
    _check(load().cube_stats_hist_minmax(C.c_void_p(ptr), _dims(dims), nbins, C.byref(out),
                                         counts.ctypes.data))
    return Stats.from_c(out), counts


def cube_stats_async(ptr: int, dims, dev_out: int, stream: int = 0) -> None:
    _check(load().cube_stats_async(C.c_void_p(ptr), _dims(dims), C.c_void_p(dev_out),
                                   C.c_void_p(stream)))


def cube_hist_async(ptr: int, dims, lo: float, hi: float, nbins: int, dev_counts: int,
                    stream: int = 0) -> None:
    _check(load().cube_hist_async(C.c_void_p(ptr), _dims(dims), lo, hi, nbins,
                                  C.c_void_p(dev_counts), C.c_void_p(stream)))


def cube_stats_hist_async(ptr: int, dims, lo: float, hi: float, nbins: int, dev_out: int,
                          dev_counts: int, stream: int = 0) -> None:
    _check(load().cube_stats_hist_async(C.c_void_p(ptr), _dims(dims), lo, hi, nbins,
                                        C.c_void_p(dev_out), C.c_void_p(dev_counts),
                                        C.c_void_p(stream)))


def cube_stats_hist_minmax_async(ptr: int, dims, nbins: int, dev_out: int, dev_counts: int,
                                 stream: int = 0) -> None:
    _check(load().cube_stats_hist_minmax_async(C.c_void_p(ptr), _dims(dims), nbins,
                                               C.c_void_p(dev_out), C.c_void_p(dev_counts),
                                               C.c_void_p(stream)))


CUBE_NOALLOC_MAX_RECORDS = 16384


def cube_stats_hist_noalloc(ptr: int, dims, lo: float, hi: float, nbins: int, dev_out: int,
                            dev_counts: int, stream: int = 0) -> None:
    """The allocation-free fused call (device outputs, stream-ordered)."""
    _check(load().cube_stats_hist_noalloc(C.c_void_p(ptr), _dims(dims), lo, hi, nbins,
                                          C.c_void_p(dev_out), C.c_void_p(dev_counts),
                                          C.c_void_p(stream)))


def cube_set_accum_mode(mode: int) -> int:
    return _check(load().cube_set_accum_mode(mode))


def cube_set_hist_mode(mode: int) -> int:
    """Histogram form of this thread's later single-box passes; returns the previous one."""
    return _check(load().cube_set_hist_mode(mode))


def cube_set_partition(chunk_log2: int) -> int:
    """Partition of this thread's later single-box passes: CUBE_PARTITION_AUTO,
    CUBE_PARTITION_STATIC, or k for a dynamic partition into chunks of 2^k
    voxels; returns the previous setting."""
    return _check(load().cube_set_partition(chunk_log2))


def cube_describe_plan(ptr: int, dims, kind: int, nbins: int = 1) -> dict:
    """The plan of this thread's next single-box pass of `kind` over the box."""
    import json
    buf = C.create_string_buffer(512)
    _check(load().cube_describe_plan(C.c_void_p(ptr), _dims(dims), kind, nbins, buf, 512))
    return json.loads(buf.value.decode())


def cube_set_launch(threads: int = 0, blocks: int = 0, hist_copies: int = 0,
                    unroll: int = 0) -> None:
    _check(load().cube_set_launch(threads, blocks, hist_copies, unroll))


def cube_select(ptr: int, dims, rank: int) -> float:
    v = C.c_float()
    _check(load().cube_select(C.c_void_p(ptr), _dims(dims), rank, C.byref(v)))
    return v.value


def cube_median(ptr: int, dims):
    """(median, n_valid) of a device box."""
    m, n = C.c_double(), C.c_uint64()
    _check(load().cube_median(C.c_void_p(ptr), _dims(dims), C.byref(m), C.byref(n)))
    return m.value, n.value


CUBE_MAX_QUANTILES = 64


def cube_quantiles(ptr: int, dims, q):
    """(float64 array of the quantiles at levels q, n_valid) of a device box."""
    qa = np.ascontiguousarray(np.atleast_1d(np.asarray(q, dtype=np.float64)))
    out = np.empty(qa.size, dtype=np.float64)
    n = C.c_uint64()
    _check(load().cube_quantiles(C.c_void_p(ptr), _dims(dims), C.c_void_p(qa.ctypes.data),
                                 qa.size, C.c_void_p(out.ctypes.data), C.byref(n)))
    return out, n.value


def quantiles(t, q):
    ptr, d = box_of(t)
    return cube_quantiles(ptr, d, q)


def cube_last_quantile_reads() -> int:
    """Reads of the box made by this thread's last successful quantiles call."""
    return int(load().cube_last_quantile_reads())


def select(t, rank: int) -> float:
    ptr, d = box_of(t)
    return cube_select(ptr, d, rank)


def median(t):
    ptr, d = box_of(t)
    return cube_median(ptr, d)


def cube_autotune(ptr: int, dims, kind: int, lo: float = 0.0, hi: float = 0.0, nbins: int = 1,
                  reps: int = 5) -> dict:
    """Tune the launch shape for one pass kind on this data; returns the
    autotuner's JSON report as a dict."""
    import json
    buf = C.create_string_buffer(1024)
    _check(load().cube_autotune(C.c_void_p(ptr), _dims(dims), kind, lo, hi, nbins, reps, buf,
                                len(buf)))
    return json.loads(buf.value.decode())


def cube_autotune_batch(queries, reps: int = 5) -> dict:
    """Tune the batched launch's automatic rule on these queries (their
    device outputs are overwritten); returns the autotuner's JSON report."""
    import json
    arr = (cube_query_t * len(queries))(*queries)
    buf = C.create_string_buffer(1024)
    _check(load().cube_autotune_batch(arr, len(queries), reps, buf, len(buf)))
    return json.loads(buf.value.decode())


def cube_tune_save(path: str) -> None:
    _check(load().cube_tune_save(path.encode()))


def cube_tune_load(path: str) -> int:
    return _check(load().cube_tune_load(path.encode()))


def cube_tune_clear() -> None:
    load().cube_tune_clear()


def cube_shutdown() -> None:
    load().cube_shutdown()


def cube_release_stream(stream: int) -> None:
    """Free the workspace the single-box calls keep for this stream."""
    load().cube_release_stream(C.c_void_p(stream))


# ------------------------------------------------------------ tensor helpers
def box_of(t) -> tuple:
    """(device address, [nx, ny, nz, sy, sz]) of a float32 CUDA tensor."""
    import torch
    if t.dtype != torch.float32:
        raise TypeError("cube tensors are float32")
    if not t.is_cuda:
        raise ValueError("cube tensors live on the GPU")
    if t.dim() == 1:
        if t.numel() > 1 and t.stride(0) != 1:
            raise ValueError("1-D cube tensors must be contiguous")
        return t.data_ptr(), [t.numel(), 1, 1, t.numel(), t.numel()]
    if t.dim() != 3:
        raise ValueError("cube tensors are 1-D or 3-D [z, y, x]")
    nz, ny, nx = t.shape
    sz, sy, sx = t.stride()
    if nx > 1 and sx != 1:
        raise ValueError("the x axis must have unit stride")
    return t.data_ptr(), [nx, ny, nz, sy if ny > 1 else nx, sz if nz > 1 else (sy if ny > 1 else nx) * ny]


def stats(t) -> Stats:
    ptr, d = box_of(t)
    return cube_stats(ptr, d[0], d[1], d[2], (d[3], d[4]))


def hist(t, lo: float, hi: float, nbins: int) -> np.ndarray:
    ptr, d = box_of(t)
    return cube_hist(ptr, d, lo, hi, nbins)


def stats_hist(t, lo: float, hi: float, nbins: int):
    ptr, d = box_of(t)
    return cube_stats_hist(ptr, d, lo, hi, nbins)


def stats_hist_minmax(t, nbins: int):
    ptr, d = box_of(t)
    return cube_stats_hist_minmax(ptr, d, nbins)


# ------------------------------------------------------------------ batches
def make_query(ptr: int, dims, kind: int, nbins: int = 0, lo: float = 0.0, hi: float = 0.0,
               out: int = 0, counts: int = 0) -> cube_query_t:
    q = cube_query_t()
    q.ptr = ptr
    d = list(dims) + [0] * (5 - len(dims))
    for i in range(5):
        q.dims[i] = d[i]
    q.kind, q.nbins, q.lo, q.hi = kind, nbins, lo, hi
    q.out, q.counts = out or None, counts or None
    return q


def cube_project(ptr: int, dims, mip: int = 0, mom0: int = 0, nvalid: int = 0,
                 stream: int = 0) -> None:
    """Projections along z into device maps (addresses; 0 = not wanted)."""
    _check(load().cube_project(C.c_void_p(ptr), _dims(dims), C.c_void_p(mip or None),
                               C.c_void_p(mom0 or None), C.c_void_p(nvalid or None),
                               C.c_void_p(stream or None)))


def project(t):
    """(mip float32 [ny, nx], mom0 float64 [ny, nx], nvalid int32-viewed uint32
    [ny, nx]) device tensors of a [z, y, x] CUDA tensor, on the current
    stream."""
    import torch
    ptr, d = box_of(t)
    nx, ny = d[0], d[1]
    mip = torch.empty((ny, nx), dtype=torch.float32, device=t.device)
    mom0 = torch.empty((ny, nx), dtype=torch.float64, device=t.device)
    nv = torch.empty((ny, nx), dtype=torch.int32, device=t.device)
    cube_project(ptr, d, mip.data_ptr(), mom0.data_ptr(), nv.data_ptr(),
                 torch.cuda.current_stream(t.device).cuda_stream)
    return mip, mom0, nv


def cube_read_probe(ptr: int, dims, nbins: int, dev_out: int, stream: int = 0) -> None:
    """OR the bit patterns of the box into the device word at dev_out, read
    in the fused pass's launch shape for nbins bins."""
    _check(load().cube_read_probe(C.c_void_p(ptr), _dims(dims), nbins, C.c_void_p(dev_out),
                                  C.c_void_p(stream or None)))


def read_probe(t, nbins: int = 1024) -> int:
    """The OR of the bit patterns of a CUDA tensor's voxels, read by the probe
    kernel on the current stream (synchronous)."""
    import torch
    ptr, d = box_of(t)
    out = torch.zeros(1, dtype=torch.int32, device=t.device)
    cube_read_probe(ptr, d, nbins, out.data_ptr(), torch.cuda.current_stream(t.device).cuda_stream)
    return int(out.cpu().numpy().view(np.uint32)[0])


def host_box_of(a) -> tuple:
    """(host address, [nx, ny, nz, sy, sz]) of a float32 numpy array (or CPU
    tensor) laid out [z, y, x] with unit x-stride."""
    if not isinstance(a, np.ndarray):
        a = a.numpy()
    if a.dtype != np.float32:
        raise TypeError("cube arrays are float32")
    if a.ndim == 1:
        if a.size > 1 and a.strides[0] != 4:
            raise ValueError("1-D cube arrays must be contiguous")
        return a.ctypes.data, [a.size, 1, 1, a.size, a.size]
    if a.ndim != 3:
        raise ValueError("cube arrays are 1-D or 3-D [z, y, x]")
    nz, ny, nx = a.shape
    if a.size == 0:
        return a.ctypes.data, [nx, ny, nz, 0, 0]
    sz, sy, sx = (s // 4 for s in a.strides)
    if nx > 1 and sx != 1:
        raise ValueError("the x axis must have unit stride")
    return a.ctypes.data, [nx, ny, nz, sy if ny > 1 else nx,
                           sz if nz > 1 else (sy if ny > 1 else nx) * ny]


def cube_host_query(ptr: int, dims, kind: int, nbins: int = 0, lo: float = 0.0,
                    hi: float = 0.0, chunk_voxels: int = 0):
    """Out-of-core query over a box in host memory: (Stats or None, counts or
    None)."""
    st = cube_stats_t()
    cnt = np.zeros(max(nbins, 0) + 3, dtype=np.uint64)
    want_stats = kind != CUBE_Q_HIST
    want_hist = kind != CUBE_Q_STATS
    q = make_query(ptr, dims, kind, nbins, lo, hi,
                   C.addressof(st) if want_stats else 0,
                   cnt.ctypes.data if want_hist else 0)
    _check(load().cube_host_query(C.byref(q), chunk_voxels))
    return (Stats.from_c(st) if want_stats else None), (cnt if want_hist else None)


def host_query(a, kind: int, nbins: int = 0, lo: float = 0.0, hi: float = 0.0,
               chunk_voxels: int = 0):
    ptr, d = host_box_of(a)
    return cube_host_query(ptr, d, kind, nbins, lo, hi, chunk_voxels)


class Batch:
    """A reusable batch (cube_batch_t): enqueue a list of cube_query_t, then
    relaunch or graph-launch it.  Outputs are the device pointers in the
    queries."""

    def __init__(self, tile_voxels: int | None = None, threads: int = 0):
        """tile_voxels: None keeps the library's default (2^20), 0 asks for
        each query's automatic size."""
        self._h = C.c_void_p()
        _check(load().cube_batch_create(C.byref(self._h)))
        if tile_voxels is not None or threads:
            tv = (1 << 20) if tile_voxels is None else tile_voxels
            _check(load().cube_batch_set_tile(self._h, tv, threads))

    def enqueue(self, queries, stream: int = 0) -> None:
        arr = (cube_query_t * len(queries))(*queries)
        self._keep = arr
        _check(load().cube_batch_enqueue(self._h, arr, len(queries), C.c_void_p(stream)))

    def set_order(self, order: int) -> None:
        _check(load().cube_batch_set_order(self._h, order))

    def query_done(self, i: int) -> bool:
        """True once query i of the last launch is complete; raises CubeError
        if it completed as failed."""
        rc = load().cube_batch_query_done(self._h, i)
        if rc < 0:
            raise CubeError(rc, last_error())
        return bool(rc)

    def relaunch(self, stream: int = 0) -> None:
        _check(load().cube_batch_relaunch(self._h, C.c_void_p(stream)))

    def graph_launch(self, stream: int = 0) -> None:
        _check(load().cube_batch_graph_launch(self._h, C.c_void_p(stream)))

    def check(self) -> None:
        _check(load().cube_batch_check(self._h))

    def close(self) -> None:
        if self._h:
            load().cube_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cube_batch_run(queries) -> None:
    arr = (cube_query_t * len(queries))(*queries)
    _check(load().cube_batch_run(arr, len(queries)))


# ------------------------------------------------------------------ server
CUBE_SERVE_BATCHED, CUBE_SERVE_PLAIN = 0, 1


class Server:
    """cube_server_t: submit queries from any thread, wait for each."""

    def __init__(self, mode: int = CUBE_SERVE_BATCHED, slots: int = 4, max_batch: int = 64,
                 max_inflight_bytes: int = 1 << 30, tile_voxels: int = 0):
        self._h = C.c_void_p()
        _check(load().cube_server_create(mode, slots, max_batch, max_inflight_bytes,
                                         tile_voxels, C.byref(self._h)))

    def submit(self, q: cube_query_t) -> int:
        i = C.c_uint64()
        _check(load().cube_server_submit(self._h, C.byref(q), C.byref(i)))
        return i.value

    def wait(self, qid: int, timeout_s: float = -1.0) -> float:
        lat = C.c_double()
        _check(load().cube_server_wait(self._h, qid, timeout_s, C.byref(lat)))
        return lat.value

    def latency(self, reset: bool = False):
        p50, p99, n = C.c_double(), C.c_double(), C.c_uint64()
        _check(load().cube_server_latency(self._h, C.byref(p50), C.byref(p99), C.byref(n),
                                          1 if reset else 0))
        return p50.value, p99.value, n.value

    def close(self) -> None:
        if self._h:
            load().cube_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
