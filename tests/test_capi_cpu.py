"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol the header declares, and rejects bad arguments before any HIP call."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import paper_1111_6661_amd as cs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cubestats.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cube_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = cs.load()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), f"{n} is declared in cubestats.h but not exported"


def test_abi_version_matches_header():
    m = re.search(r"#define CUBE_ABI_VERSION (\d+)", open(HEADER).read())
    assert cs.load().cube_abi_version() == int(m.group(1))


def test_stats_struct_layout_matches_header():
    text = open(HEADER).read()
    assert "} cube_stats_t; /* 64 bytes */" in text
    assert C.sizeof(cs.cube_stats_t) == 64
    fields = [f[0] for f in cs.cube_stats_t._fields_]
    assert fields == ["n_total", "n_valid", "n_nan", "min", "max", "mean", "m2", "std",
                      "flags", "reserved"]


def _code(fn, *a):
    try:
        fn(*a)
    except cs.CubeError as e:
        return e.code, str(e)
    return 0, ""


@pytest.mark.parametrize("lo,hi,nbins,why", [
    (0.0, 1.0, 0, "nbins"), (0.0, 1.0, 65537, "nbins"), (math.nan, 1.0, 16, "NaN"),
    (0.0, math.nan, 16, "NaN"), (2.0, 1.0, 16, "hi < lo"), (-math.inf, 1.0, 16, "infinite"),
    (0.0, math.inf, 16, "infinite"), (-3e38, 3e38, 16, "overflows"), (0.0, 1e-45, 256, "narrow"),
])
def test_bad_ranges_rejected_before_gpu(lo, hi, nbins, why):
    code, msg = _code(cs.cube_hist, 0x1000, [4, 4, 4, 0, 0], lo, hi, nbins)
    assert code == cs.CUBE_EINVAL and why in msg
    code, msg = _code(cs.cube_stats_hist, 0x1000, [4, 4, 4, 0, 0], lo, hi, nbins)
    assert code == cs.CUBE_EINVAL and why in msg


@pytest.mark.parametrize("dims,why", [
    ([-1, 4, 4, 0, 0], "negative"), ([8, 4, 4, 7, 0], "row pitch"),
    ([8, 4, 4, 8, 20], "plane pitch"), ([1 << 41, 1, 1, 0, 0], "too large"),
    # pitches whose extent would wrap 64-bit arithmetic (the end of the box
    # would then look like a few bytes past its start)
    ([1, 3, 1, 3 << 61, 0], "too large"), ([1, 3, 1, (1 << 63) - 1, 0], "too large"),
    ([1, 1, 3, 0, 3 << 61], "overflows"), ([4, 2, 3, 1 << 40, 1 << 61], "overflows"),
    ([4, 1 << 22, 1, 1 << 41, 0], "too large"), ([1, 2, 2, 1 << 61, 0], "overflows"),
])
def test_bad_shapes_rejected_before_gpu(dims, why):
    code, msg = _code(cs.cube_hist, 0x1000, dims, 0.0, 1.0, 8)
    assert code == cs.CUBE_EINVAL and why in msg


def test_bad_pointers_rejected_before_gpu():
    code, msg = _code(cs.cube_stats, 0, 4, 4, 4)
    assert code == cs.CUBE_EINVAL and "NULL" in msg
    code, msg = _code(cs.cube_stats, 0x1002, 4, 4, 4)
    assert code == cs.CUBE_EINVAL and "aligned" in msg
    lib = cs.load()
    d = (C.c_int64 * 5)(4, 4, 4, 0, 0)
    assert lib.cube_stats_hist(C.c_void_p(0x1000), d, 0.0, 1.0, 8, None, None) == cs.CUBE_EINVAL
    assert lib.cube_hist(C.c_void_p(0x1000), None, 0.0, 1.0, 8, None) == cs.CUBE_EINVAL
    assert lib.cube_stats_async(C.c_void_p(0x1000), d, None, None) == cs.CUBE_EINVAL
    # the allocation-free call checks its arguments before any HIP call too
    assert lib.cube_stats_hist_noalloc(C.c_void_p(0x1000), d, 0.0, 1.0, 8, None, None,
                                       None) == cs.CUBE_EINVAL
    code, msg = _code(cs.cube_stats_hist_noalloc, 0x1002, [4, 4, 4, 0, 0], 0.0, 1.0, 8, 0x2000,
                      0x3000)
    assert code == cs.CUBE_EINVAL and "aligned" in msg
    code, msg = _code(cs.cube_stats_hist_noalloc, 0x1000, [4, 4, 4, 0, 0], 1.0, 0.0, 8, 0x2000,
                      0x3000)
    assert code == cs.CUBE_EINVAL and "hi < lo" in msg


def test_mode_and_launch_setters_validate():
    assert _code(cs.cube_set_accum_mode, 7)[0] == cs.CUBE_EINVAL
    assert _code(cs.cube_set_launch, 100, 0, 0)[0] == cs.CUBE_EINVAL
    assert _code(cs.cube_set_launch, 256, 5000, 0)[0] == cs.CUBE_EINVAL
    assert _code(cs.cube_set_launch, 256, 0, 3)[0] == cs.CUBE_EINVAL
    prev = cs.cube_set_accum_mode(cs.CUBE_ACCUM_KAHAN32)
    assert cs.cube_set_accum_mode(prev) == cs.CUBE_ACCUM_KAHAN32
    cs.cube_set_launch(0, 0, 0, 0)
    assert _code(cs.cube_set_hist_mode, 3)[0] == cs.CUBE_EINVAL
    assert _code(cs.cube_set_hist_mode, -1)[0] == cs.CUBE_EINVAL
    assert cs.cube_set_hist_mode(cs.CUBE_HIST_HOT) == cs.CUBE_HIST_AUTO
    assert cs.cube_set_hist_mode(cs.CUBE_HIST_PLAIN) == cs.CUBE_HIST_HOT
    assert cs.cube_set_hist_mode(cs.CUBE_HIST_AUTO) == cs.CUBE_HIST_PLAIN
    for bad in (-1, 2, cs.CUBE_CHUNK_LOG2_MIN - 1, cs.CUBE_CHUNK_LOG2_MAX + 1):
        assert _code(cs.cube_set_partition, bad)[0] == cs.CUBE_EINVAL
    assert cs.cube_set_partition(18) == cs.CUBE_PARTITION_AUTO
    assert cs.cube_set_partition(cs.CUBE_PARTITION_STATIC) == 18
    assert cs.cube_set_partition(cs.CUBE_PARTITION_AUTO) == cs.CUBE_PARTITION_STATIC


def test_describe_plan_rejects_bad_arguments_before_gpu():
    buf = C.create_string_buffer(256)
    d = (C.c_int64 * 5)(8, 1, 1, 0, 0)
    lib = cs.load()
    assert lib.cube_describe_plan(C.c_void_p(0x1000), d, 7, 16, buf, 256) == cs.CUBE_EINVAL
    assert lib.cube_describe_plan(C.c_void_p(0x1000), d, cs.CUBE_Q_FUSED, 0, buf, 256) == \
        cs.CUBE_EINVAL
    assert lib.cube_describe_plan(C.c_void_p(0x1000), d, cs.CUBE_Q_FUSED, 16, None, 256) == \
        cs.CUBE_EINVAL
    assert "kind" in cs.last_error() or "NULL" in cs.last_error()


def test_mode_is_per_thread():
    """The precision mode set on one thread is not seen by another: a new
    thread starts from the production mode, whatever the caller set."""
    import threading
    prev = cs.cube_set_accum_mode(cs.CUBE_ACCUM_NAIVE32)
    seen = []
    try:
        th = threading.Thread(target=lambda: seen.append(
            cs.cube_set_accum_mode(cs.CUBE_ACCUM_KAHAN32)))
        th.start()
        th.join()
        assert seen == [cs.CUBE_ACCUM_FP64MERGE]
        # the other thread's KAHAN32 did not reach this one
        assert cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE) == cs.CUBE_ACCUM_NAIVE32
    finally:
        cs.cube_set_accum_mode(prev)


def test_binding_has_no_cpu_fallback():
    """The tensor helpers refuse CPU tensors instead of computing on the CPU."""
    import torch
    with pytest.raises(ValueError):
        cs.stats(torch.zeros(8))
    src = open(os.path.join(ROOT, "paper_1111_6661_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_tuning_table_round_trip(tmp_path):
    """The shipped gfx950 table loads; save writes what load reads back; bad
    files are rejected without touching the table (no GPU call involved)."""
    table = os.path.join(ROOT, "paper_1111_6661_amd", "tuning", "gfx950.json")
    cs.cube_tune_clear()
    try:
        n = cs.cube_tune_load(table)
        assert n >= 3
        out = tmp_path / "t.json"
        cs.cube_tune_save(str(out))
        cs.cube_tune_clear()
        assert cs.cube_tune_load(str(out)) == n
        lines = sorted(l.strip().rstrip(",") for l in open(out) if '"kind"' in l)
        want = sorted(l.strip().rstrip(",") for l in open(table) if '"kind"' in l)
        assert [l.split('"ms"')[0] for l in lines] == [l.split('"ms"')[0] for l in want]
        bad_arch = tmp_path / "arch.json"
        bad_arch.write_text(open(table).read().replace("gfx950", "gfx942"))
        with pytest.raises(cs.CubeError):
            cs.cube_tune_load(str(bad_arch))
        bad_entry = tmp_path / "entry.json"
        bad_entry.write_text(open(table).read().replace('"unroll": 4', '"unroll": 3', 1))
        with pytest.raises(cs.CubeError):
            cs.cube_tune_load(str(bad_entry))
        with pytest.raises(cs.CubeError):
            cs.cube_tune_load(str(tmp_path / "missing.json"))
        # the optional hot-bin field: 0 or 1 round-trips, anything else is refused
        hot = tmp_path / "hot.json"
        hot.write_text('{"arch": "gfx950", "entries": [\n  {"kind": 2, "bins_log2": 12, '
                       '"size_log2": 35, "threads": 1024, "unroll": 4, "copies": 8, '
                       '"blocks_per_cu": 2, "ms": 1.0, "hot": 1}\n]}\n')
        cs.cube_tune_clear()
        assert cs.cube_tune_load(str(hot)) == 1
        cs.cube_tune_save(str(out))
        assert '"hot": 1' in open(out).read()
        # the batched launch's rule: one line, round-trips, bad values refused
        rule = tmp_path / "rule.json"
        rule.write_text('{"arch": "gfx950", "entries": [\n  {"kind": 4, "batch_threads": 256, '
                        '"unroll": 2, "floor_log2": 17, "cap_log2": 20, "tiles_log2": 10, "lds_kib": 128, '
                        '"ms": 0.25}\n]}\n')
        cs.cube_tune_clear()
        assert cs.cube_tune_load(str(rule)) == 1
        cs.cube_tune_save(str(out))
        assert '"batch_threads": 256, "unroll": 2, "floor_log2": 17, "cap_log2": 20, "tiles_log2": 10, ' \
               '"lds_kib": 128' in open(out).read()
        for bad in ('"batch_threads": 300', '"unroll": 3', '"cap_log2": 16', '"lds_kib": 200'):
            key = bad.split(":")[0]
            txt = open(rule).read()
            i = txt.index(key)
            j = txt.index(",", i)
            (tmp_path / "badrule.json").write_text(txt[:i] + bad + txt[j:])
            with pytest.raises(cs.CubeError):
                cs.cube_tune_load(str(tmp_path / "badrule.json"))
        bad_hot = tmp_path / "badhot.json"
        bad_hot.write_text(open(hot).read().replace('"hot": 1', '"hot": 2'))
        with pytest.raises(cs.CubeError):
            cs.cube_tune_load(str(bad_hot))
        # the optional partition field: a chunk size round-trips; sizes outside
        # the allowed range, and a dynamic partition with the hot-bin form, are refused
        dyn = tmp_path / "dyn.json"
        dyn.write_text(open(hot).read().replace('"hot": 1', '"hot": 0, "chunk_log2": 19'))
        cs.cube_tune_clear()
        assert cs.cube_tune_load(str(dyn)) == 1
        cs.cube_tune_save(str(out))
        assert '"hot": 0, "chunk_log2": 19' in open(out).read()
        for bad in ('"hot": 0, "chunk_log2": 11', '"hot": 0, "chunk_log2": 27',
                    '"hot": 1, "chunk_log2": 19'):
            (tmp_path / "baddyn.json").write_text(
                open(dyn).read().replace('"hot": 0, "chunk_log2": 19', bad))
            with pytest.raises(cs.CubeError):
                cs.cube_tune_load(str(tmp_path / "baddyn.json"))
    finally:
        cs.cube_tune_clear()


@pytest.mark.parametrize("q,why", [([], "m=0"), ([0.5] * 65, "m=65"), ([1.5], "outside [0, 1]"),
                                   ([-0.25], "outside [0, 1]"), ([math.nan], "outside [0, 1]")])
def test_bad_quantile_levels_rejected_before_gpu(q, why):
    code, msg = _code(cs.cube_quantiles, 0x1000, [4, 4, 4, 0, 0], q)
    assert code == cs.CUBE_EINVAL and why in msg


def test_quantile_and_probe_boxes_rejected_before_gpu():
    code, msg = _code(cs.cube_quantiles, 0, [4, 4, 4, 0, 0], [0.5])
    assert code == cs.CUBE_EINVAL and "NULL" in msg
    code, msg = _code(cs.cube_quantiles, 0x1000, [8, 4, 4, 7, 0], [0.5])
    assert code == cs.CUBE_EINVAL and "row pitch" in msg
    for nbins, why in ((0, "nbins"), (65537, "nbins")):
        code, msg = _code(cs.cube_read_probe, 0x1000, [4, 4, 4, 0, 0], nbins, 0x2000)
        assert code == cs.CUBE_EINVAL and why in msg
    code, msg = _code(cs.cube_read_probe, 0x1000, [4, 4, 4, 0, 0], 16, 0)
    assert code == cs.CUBE_EINVAL and "NULL" in msg
    code, msg = _code(cs.cube_read_probe, 0x1000, [4, 4, 4, 0, 0], 16, 0x2002)
    assert code == cs.CUBE_EINVAL and "aligned" in msg
    code, msg = _code(cs.cube_read_probe, 0, [4, 4, 4, 0, 0], 16, 0x2000)
    assert code == cs.CUBE_EINVAL and "NULL" in msg
