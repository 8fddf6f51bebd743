"""Out-of-core queries over cubes in host memory (GPU) against the oracle.

The chunk sizes are small so that every cube here crosses many chunks, with
ragged last chunks, rows split across chunks and strided host views.
"""
import numpy as np
import pytest

import oracle
from tests.parity import assert_counts_match, assert_stats_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    return cs


@pytest.fixture(scope="module")
def cube():
    import synth
    r = synth.WORKLOADS["tiny"].scaled(203, 150, 37)
    return synth.make_numpy(r, 31)


def check_kinds(cs, a, chunk, nbins=200, lo=-2.5, hi=20.0, what=""):
    ref = oracle.stats(a)
    st, _ = cs.host_query(a, cs.CUBE_Q_STATS, chunk_voxels=chunk)
    assert_stats_match(st, ref, f"stats {what}")
    _, cnt = cs.host_query(a, cs.CUBE_Q_HIST, nbins, lo, hi, chunk_voxels=chunk)
    want = oracle.hist(a, lo, hi, nbins)
    assert_counts_match(cnt, want, f"hist {what}")
    st, cnt = cs.host_query(a, cs.CUBE_Q_FUSED, nbins, lo, hi, chunk_voxels=chunk)
    assert_stats_match(st, ref, f"fused {what}")
    assert_counts_match(cnt, want, f"fused counts {what}")
    if ref.n_valid:
        st, cnt = cs.host_query(a, cs.CUBE_Q_MINMAX, nbins, chunk_voxels=chunk)
        assert_stats_match(st, ref, f"minmax {what}")
        assert_counts_match(cnt, oracle.hist(a, ref.min, ref.max, nbins), f"minmax counts {what}")


@pytest.mark.parametrize("chunk", [1 << 12, 5001, 1 << 16, 0])
def test_host_chunks(cs, cube, chunk):
    check_kinds(cs, cube, chunk, what=f"chunk {chunk}")


def test_host_strided_view_and_long_rows(cs, cube):
    view = cube[3:30, 7:140, 5:199]
    check_kinds(cs, view, 1 << 12, what="strided view")
    # rows longer than a chunk: a single long row, and 2-D rows of 10^4
    row = np.ascontiguousarray(cube.reshape(-1)[:100_003])
    check_kinds(cs, row, 1 << 12, what="one long row")
    rows = np.ascontiguousarray(cube.reshape(-1)[:5 * 10_000]).reshape(1, 5, 10_000)
    check_kinds(cs, rows[:, :, 3:9_999], 1 << 12, what="strided long rows")


def test_host_pinned_equals_resident(cs, cube):
    pinned = torch.empty(cube.shape, dtype=torch.float32, pin_memory=True)
    pinned.copy_(torch.from_numpy(cube))
    dev = pinned.cuda()
    st_h, cnt_h = cs.host_query(pinned, cs.CUBE_Q_FUSED, 256, -2.5, 20.0, chunk_voxels=1 << 14)
    st_d, cnt_d = cs.stats_hist(dev, -2.5, 20.0, 256)
    assert np.array_equal(cnt_h, cnt_d)
    assert st_h.n_valid == st_d.n_valid and st_h.min == st_d.min and st_h.max == st_d.max
    assert_stats_match(st_h, oracle.stats(cube), "pinned")


def test_host_special_cases(cs):
    empty = np.zeros((0, 4, 4), np.float32)
    st, cnt = cs.host_query(empty, cs.CUBE_Q_FUSED, 8, 0.0, 1.0)
    assert st.n_total == 0 and st.flags & cs.CUBE_NO_VALID and not cnt.any()
    nan = np.full(10_000, np.nan, np.float32)
    st, cnt = cs.host_query(nan, cs.CUBE_Q_MINMAX, 16, chunk_voxels=1 << 12)
    assert st.n_valid == 0 and st.n_nan == 10_000
    assert int(cnt[16 + 2]) == 10_000 and not cnt[:18].any()
    # chunks where every voxel is blank, between valid ones
    a = np.arange(3 * 8192, dtype=np.float32)
    a[4096:12288] = np.nan
    check_kinds(cs, a, 1 << 12, nbins=64, lo=0.0, hi=30000.0, what="blank chunks")
    on_device = torch.zeros(100, device="cuda")
    with pytest.raises(cs.CubeError):
        cs.cube_host_query(on_device.data_ptr(), [100, 1, 1, 100, 100], cs.CUBE_Q_STATS)
    with pytest.raises(cs.CubeError):
        cs.host_query(nan, cs.CUBE_Q_STATS, chunk_voxels=100)
    with pytest.raises(cs.CubeError):
        cs.host_query(a, cs.CUBE_Q_HIST, 64, 1.0, 0.0)


def test_host_pageable_staging_large(cs):
    """Pageable sources go through pinned staging buffers, gathered by several
    host threads: a strided view whose planes (about 10^6 voxels, rows at a
    pitch) fill a chunk each, and one row longer than a staged chunk (2^24
    voxels), with default chunk sizes; the same arrays pinned give the same
    counts and extrema."""
    rng = np.random.default_rng(77)
    full = (rng.standard_normal((8, 1024, 1024)) * 4 + 1).astype(np.float32)
    full[rng.random(full.shape) < 0.01] = np.nan
    view = full[1:8, 5:1000, 3:1020]
    check_kinds(cs, view, 0, nbins=300, lo=-10.0, hi=12.0, what="large strided view")
    row = (rng.standard_normal((1 << 24) + 12345) * 2).astype(np.float32)
    row[::977] = np.nan
    check_kinds(cs, row, 0, nbins=64, lo=-6.0, hi=6.0, what="row over two staged chunks")
    pinned = torch.from_numpy(row).pin_memory()
    st_p, cnt_p = cs.host_query(pinned, cs.CUBE_Q_FUSED, 64, -6.0, 6.0)
    st_s, cnt_s = cs.host_query(row, cs.CUBE_Q_FUSED, 64, -6.0, 6.0)
    assert np.array_equal(cnt_p, cnt_s)
    assert st_p.min == st_s.min and st_p.max == st_s.max and st_p.n_valid == st_s.n_valid
