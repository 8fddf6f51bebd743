"""The allocation-free fused call against the allocating one, through the C ABI.

cube_stats_hist_noalloc keeps its scratch in one static device array per
device instead of a per-stream workspace.  Two calls in a row, the second on a
smaller strided box with fewer bins, must each give what cube_stats_hist_async
gives on the same input: counts and extrema bit-exact, and, since both run the
same kernel on the same grid, the moments too.  A grid narrowed to the
scratch's record limit (a tuned shape wider than it) must still match to the
oracle's bar, and an explicit shape beyond the limit is refused.
"""
import numpy as np
import pytest

import oracle
from tests.parity import assert_counts_match, assert_stats_match, same_f32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    return cs


def outputs(nbins):
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    counts = torch.zeros(nbins + 3, dtype=torch.int64, device="cuda")
    return out, counts


def read(cs, out, counts):
    st = cs.Stats.from_bytes(out.cpu().numpy().tobytes())
    return st, counts.cpu().numpy().view(np.uint64)


def run_both(cs, t, lo, hi, nbins):
    """(allocating call's results, allocation-free call's results)."""
    ptr, d = cs.box_of(t)
    stream = torch.cuda.current_stream().cuda_stream
    o1, c1 = outputs(nbins)
    cs.cube_stats_hist_async(ptr, d, lo, hi, nbins, o1.data_ptr(), c1.data_ptr(), stream)
    o2, c2 = outputs(nbins)
    # poison the outputs: everything the call reports must be written by it
    o2.fill_(0xA5)
    c2.fill_(-1)
    cs.cube_stats_hist_noalloc(ptr, d, lo, hi, nbins, o2.data_ptr(), c2.data_ptr(), stream)
    torch.cuda.synchronize()
    return read(cs, o1, c1), read(cs, o2, c2)


def assert_same(a, b, what):
    (sa, ca), (sb, cb) = a, b
    assert_counts_match(cb, ca, what + " counts")
    for f in ("n_total", "n_valid", "n_nan", "flags"):
        assert getattr(sb, f) == getattr(sa, f), (what, f, getattr(sb, f), getattr(sa, f))
    assert same_f32(sb.min, sa.min) and same_f32(sb.max, sa.max), what
    for f in ("mean", "m2", "std"):
        assert np.array_equal(np.float64(getattr(sb, f)), np.float64(getattr(sa, f)),
                              equal_nan=True), (what, f, getattr(sb, f), getattr(sa, f))


def make_cube(nx, ny, nz, seed):
    import synth
    r = synth.Recipe(nx=nx, ny=ny, nz=nz, n_sources=12, p_voxel_nan=0.01)
    return synth.cube_tensor(r, seed, device="cuda")


def test_two_calls_in_a_row_match_the_allocating_call(cs):
    big = make_cube(1000, 517, 66, 7)            # 34.1M voxels, ragged rows
    host = big.cpu().numpy()
    ref = oracle.stats(host)
    lo, hi, nb = float(ref.min), float(ref.max), 4096
    a, b = run_both(cs, big, lo, hi, nb)
    assert_same(a, b, "first call")
    assert_stats_match(b[0], ref, "first call vs oracle")
    assert_counts_match(b[1], oracle.hist(host, lo, hi, nb), "first call vs oracle")

    # second call: a smaller strided sub-box with fewer bins and its own range
    sub = big[3:40, 11:300, 5:770]
    sh = sub.cpu().numpy()
    sref = oracle.stats(sh)
    lo2, hi2, nb2 = -1.5, 9.25, 100
    a2, b2 = run_both(cs, sub, lo2, hi2, nb2)
    assert_same(a2, b2, "second call")
    assert_stats_match(b2[0], sref, "second call vs oracle")
    assert_counts_match(b2[1], oracle.hist(sh, lo2, hi2, nb2), "second call vs oracle")


def test_empty_and_tiny_boxes(cs):
    t = make_cube(37, 3, 2, 9)
    h = t.cpu().numpy()
    ref = oracle.stats(h)
    a, b = run_both(cs, t, float(ref.min), float(ref.max), 7)
    assert_same(a, b, "tiny")
    e = t[:0]
    a, b = run_both(cs, e, 0.0, 1.0, 7)
    assert_same(a, b, "empty")
    assert b[0].n_total == 0 and b[1].sum() == 0


def test_narrowed_grid_and_refused_shape(cs, tmp_path):
    t = make_cube(512, 512, 40, 11)               # 10.5M voxels: size class 2^24
    h = t.cpu().numpy()
    ref = oracle.stats(h)
    lo, hi, nb = float(ref.min), float(ref.max), 512
    # a tuned shape wider than the scratch: 1024-thread blocks, 64 per CU
    # (4096 blocks after the planner's cap, 65536 wave records)
    table = tmp_path / "wide.json"
    table.write_text('{"arch": "gfx950", "entries": [\n'
                     '  {"kind": 2, "bins_log2": 9, "size_log2": 24, "threads": 1024, '
                     '"unroll": 4, "copies": 8, "blocks_per_cu": 64, "ms": 1.0}\n]}\n')
    try:
        cs.cube_tune_clear()
        assert cs.cube_tune_load(str(table)) == 1
        a, b = run_both(cs, t, lo, hi, nb)
        assert_counts_match(b[1], a[1], "narrowed counts")
        assert_counts_match(b[1], oracle.hist(h, lo, hi, nb), "narrowed vs oracle")
        assert_stats_match(b[0], ref, "narrowed vs oracle")
        assert_stats_match(a[0], ref, "wide grid vs oracle")
    finally:
        cs.cube_tune_clear()
    # an explicit grid beyond the records the scratch holds is refused
    ptr, d = cs.box_of(t)
    o, c = outputs(nb)
    cs.cube_set_launch(1024, 4096, 0, 0)
    try:
        with pytest.raises(cs.CubeError) as ei:
            cs.cube_stats_hist_noalloc(ptr, d, lo, hi, nb, o.data_ptr(), c.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
        assert ei.value.code == cs.CUBE_EINVAL and "wave records" in str(ei.value)
    finally:
        cs.cube_set_launch(0, 0, 0, 0)
