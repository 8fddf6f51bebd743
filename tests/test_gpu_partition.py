"""The dynamic partition of the single-box pass against the oracle.

With cube_set_partition(k) the box is cut into chunks of about 2^k voxels
that a resident wave of blocks claims at run time; every chunk gets one FP64
record and the records are merged in chunk order.  Results must meet the
same parity bar as the static partition (counts, n_valid and extrema
bit-exact, moments within tests/parity.py's bound), must not depend on the
grid or on which block took which chunk, and the histogram counts must equal
the static partition's exactly.
"""
import numpy as np
import pytest

import oracle
from tests.parity import assert_counts_match, assert_stats_match
from tests.test_gpu_parity import check_all

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    yield cs
    cs.cube_set_partition(cs.CUBE_PARTITION_AUTO)
    cs.cube_set_launch(0, 0, 0, 0)


@pytest.fixture(scope="module")
def tiny():
    import synth
    r = synth.WORKLOADS["tiny"]
    t = synth.cube_tensor(r, synth.BASE_SEED, device="cuda")
    return t, t.cpu().numpy()


class partition:
    def __init__(self, cs, k):
        self.cs, self.k = cs, k

    def __enter__(self):
        self.prev = self.cs.cube_set_partition(self.k)

    def __exit__(self, *exc):
        self.cs.cube_set_partition(self.prev)


@pytest.mark.parametrize("k", [12, 14, 17])
def test_tiny_workload(cs, tiny, k):
    t, host = tiny
    ref = oracle.stats(host)
    with partition(cs, k):
        check_all(cs, t, host, 256, f"tiny k={k}")
        lo = float(np.float32(ref.mean - 2 * ref.std))
        hi = float(np.float32(ref.mean + 2 * ref.std))
        check_all(cs, t, host, 256, f"tiny-2sigma k={k}", lo, hi)
        for nb in (1, 1000, 65536):
            check_all(cs, t, host, nb, f"tiny-{nb}bins k={k}")


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (1_000_003, 1, 1), (257, 129, 33),
                                   (17, 1, 900), (63, 65, 64)])
def test_ragged_shapes(cs, shape):
    import synth
    nx, ny, nz = shape
    r = synth.WORKLOADS["tiny"].scaled(nx, ny, nz)
    t = synth.cube_tensor(r, 1234 + nx, device="cuda")
    with partition(cs, 12):
        check_all(cs, t, t.cpu().numpy(), 128, f"shape{shape}")


@pytest.mark.parametrize("box", [np.s_[3:40, 5:60, 7:200], np.s_[10:11, :, 1:255],
                                 np.s_[5:60, 0:64, 33:34]])
def test_strided_sub_boxes(cs, box):
    import synth
    r = synth.WORKLOADS["tiny"].scaled(256, 64, 64)
    big = synth.cube_tensor(r, 4242, device="cuda")
    view = big[box]
    with partition(cs, 12):
        check_all(cs, view, big.cpu().numpy()[box], 64, f"box{box}")


@pytest.mark.parametrize("threads,unroll", [(256, 4), (1024, 2)])
def test_results_independent_of_grid(cs, tiny, threads, unroll):
    """Same chunks and block shape, any grid: bit-identical results."""
    t, host = tiny
    ref = oracle.stats(host)
    got = []
    with partition(cs, 12):
        for blocks in (1, 3, 64, 0):
            cs.cube_set_launch(threads, blocks, 8, unroll)
            try:
                got.append((cs.stats(t), cs.stats_hist(t, ref.min, ref.max, 512),
                            cs.hist(t, -2.0, 30.0, 300)))
            finally:
                cs.cube_set_launch(0, 0, 0, 0)
    for g in got[1:]:
        assert g[0] == got[0][0]
        assert g[1][0] == got[0][1][0]
        assert np.array_equal(g[1][1], got[0][1][1])
        assert np.array_equal(g[2], got[0][2])
    assert_stats_match(got[0][0], ref, "grid-independent")


def test_counts_equal_static(cs, tiny):
    t, host = tiny
    ref = oracle.stats(host)
    with partition(cs, cs.CUBE_PARTITION_STATIC):
        st0, c0 = cs.stats_hist(t, ref.min, ref.max, 4096)
    for k in (12, 16):
        with partition(cs, k):
            st, c = cs.stats_hist(t, ref.min, ref.max, 4096)
        assert np.array_equal(c, c0), k
        assert (st.n_valid, st.min, st.max) == (st0.n_valid, st0.min, st0.max)
        assert abs(st.mean - st0.mean) <= 1e-9 * max(1.0, abs(st0.mean))


def test_other_accumulation_modes_keep_the_static_partition(cs, tiny):
    """The dynamic pass accumulates FP64MERGE moments only: under another mode
    the setting changes nothing, bit for bit."""
    t, host = tiny
    for mode in (cs.CUBE_ACCUM_KAHAN32, cs.CUBE_ACCUM_NAIVE32):
        prev = cs.cube_set_accum_mode(mode)
        try:
            with partition(cs, cs.CUBE_PARTITION_STATIC):
                a = cs.stats_hist(t, -2.0, 30.0, 256)
            with partition(cs, 12):
                b = cs.stats_hist(t, -2.0, 30.0, 256)
        finally:
            cs.cube_set_accum_mode(prev)
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1])


def test_hot_bin_form_keeps_the_static_partition(cs, tiny):
    t, host = tiny
    ref = oracle.stats(host)
    want = oracle.hist(host, ref.min, ref.max, 256)
    prev = cs.cube_set_hist_mode(cs.CUBE_HIST_HOT)
    try:
        with partition(cs, 12):
            st, c = cs.stats_hist(t, ref.min, ref.max, 256)
    finally:
        cs.cube_set_hist_mode(prev)
    assert_counts_match(c, want, "hot under a dynamic setting")
    assert_stats_match(st, ref, "hot under a dynamic setting")


def test_probe_reads_every_voxel(cs, tiny):
    t, host = tiny
    want = int(np.bitwise_or.reduce(host.reshape(-1).view(np.uint32)))
    with partition(cs, 12):
        assert cs.read_probe(t) == want
        assert cs.read_probe(t) == want   # the chunk counter is back at 0
    with partition(cs, cs.CUBE_PARTITION_STATIC):
        assert cs.read_probe(t) == want


def test_noalloc_matches_the_allocating_call(cs, tiny):
    """Same chunk count on both paths: bit-identical results."""
    t, host = tiny
    ptr, d = cs.box_of(t)
    nb = 512
    with partition(cs, 12):
        ref_st, ref_c = cs.stats_hist(t, -2.0, 30.0, nb)
        out = torch.zeros(64, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(nb + 3, dtype=torch.int64, device="cuda")
        s = torch.cuda.current_stream()
        cs.cube_stats_hist_noalloc(ptr, d, -2.0, 30.0, nb, out.data_ptr(), cnt.data_ptr(),
                                   s.cuda_stream)
        torch.cuda.synchronize()
    assert cs.Stats.from_bytes(out.cpu().numpy().tobytes()) == ref_st
    assert np.array_equal(cnt.cpu().numpy().view(np.uint64), ref_c)


def test_lds_counters_flushed_within_a_long_block(cs):
    """One block over 34 chunks of 2^26 voxels: its LDS counters are flushed
    and cleared after 32 chunks (before any 32-bit slot could pass 2^31), and
    the counts still equal the static partition's."""
    import dataclasses

    import synth
    n = 34 << 26
    r = dataclasses.replace(synth.WORKLOADS["tiny"], nx=2048, ny=2048, nz=544, n_sources=50)
    assert r.n == n
    t = synth.cube_tensor(r, 77, device="cuda")
    with partition(cs, cs.CUBE_PARTITION_STATIC):
        st0, c0 = cs.stats_hist(t, -4.0, 8.0, 64)
    with partition(cs, 26):
        cs.cube_set_launch(1024, 1, 8, 4)
        try:
            st, c = cs.stats_hist(t, -4.0, 8.0, 64)
        finally:
            cs.cube_set_launch(0, 0, 0, 0)
    del t
    torch.cuda.empty_cache()
    assert int(c.sum()) == n
    assert np.array_equal(c, c0)
    assert (st.n_valid, st.min, st.max) == (st0.n_valid, st0.min, st0.max)
    assert abs(st.mean - st0.mean) <= 1e-9 * max(1.0, abs(st0.mean))
    assert abs(st.std - st0.std) <= 1e-7 * st0.std


def test_plan_descriptions(cs, tiny):
    t, _ = tiny
    ptr, d = cs.box_of(t)
    with partition(cs, 12):
        p = cs.cube_describe_plan(ptr, d, cs.CUBE_Q_FUSED, 256)
        assert p["partition"] == "dynamic" and p["chunks"] == t.numel() >> 12
        assert p["units"] >= p["chunks"] >= p["blocks"] >= 1
        assert p["hist"] == "lds"
        prev = cs.cube_set_accum_mode(cs.CUBE_ACCUM_KAHAN32)
        try:
            assert cs.cube_describe_plan(ptr, d, cs.CUBE_Q_FUSED, 256)["partition"] == "static"
        finally:
            cs.cube_set_accum_mode(prev)
    with partition(cs, cs.CUBE_PARTITION_STATIC):
        p = cs.cube_describe_plan(ptr, d, cs.CUBE_Q_STATS)
        assert p["partition"] == "static" and p["chunks"] == 0 and p["hist"] == "none"
    assert cs.cube_describe_plan(ptr, d, cs.CUBE_Q_HIST, 40000)["hist"] == "global"


def test_automatic_partition_by_box_size(cs):
    """Without a tuning entry, histogram passes over 2^27 voxels and more use
    chunks of 2^18 voxels, smaller boxes the static partition; an explicit
    launch shape keeps the static partition."""
    cs.cube_tune_clear()
    big = torch.empty(1 << 27, dtype=torch.float32, device="cuda")
    ptr, _ = cs.box_of(big)
    p = cs.cube_describe_plan(ptr, (1 << 27, 1, 1), cs.CUBE_Q_FUSED, 1024)
    assert p["partition"] == "dynamic" and p["chunks"] == 1 << 9, p
    p = cs.cube_describe_plan(ptr, ((1 << 27) - 4096, 1, 1), cs.CUBE_Q_HIST, 1024)
    assert p["partition"] == "static", p
    assert cs.cube_describe_plan(ptr, (1 << 27, 1, 1), cs.CUBE_Q_STATS)["partition"] == "static"
    cs.cube_set_launch(1024, 0, 0, 0)
    try:
        p = cs.cube_describe_plan(ptr, (1 << 27, 1, 1), cs.CUBE_Q_FUSED, 1024)
        assert p["partition"] == "static", p
    finally:
        cs.cube_set_launch(0, 0, 0, 0)
    del big


def _selection_arrays():
    import synth
    rng = np.random.default_rng(17)
    many = np.full(1 << 25, 1.5, np.float32)         # a bucket larger than every region
    many[::7] = rng.standard_normal(many[::7].size).astype(np.float32)
    skew = rng.standard_normal(20_000_000).astype(np.float32)
    skew[:10_000_000] = 0.25                          # one block's region overflows
    spread = (rng.standard_normal(5_000_003) * 100).astype(np.float32)
    spread[rng.random(spread.size) < 0.01] = np.nan   # the candidate path
    wide = (np.exp2(rng.uniform(-60, 60, 300_000)) * rng.choice([-1, 1], 300_000)
            ).astype(np.float32)
    wide[rng.random(wide.size) < 0.02] = np.nan      # 64 levels in dozens of top buckets
    tiny = synth.cube_tensor(synth.WORKLOADS["tiny"], synth.BASE_SEED, device="cuda")
    return {"many": many, "skew": skew, "spread": spread, "wide": wide,
            "tiny": tiny.cpu().numpy()}


@pytest.mark.parametrize("k", [12, 16])
def test_selection_median_quantiles(cs, k):
    """Selection, median and quantiles count exactly, so any partition gives
    the oracle's values bit for bit (the candidate regions and their
    overflow fallback included)."""
    from tests.parity import same_f32
    levels = [0.0, 0.1, 0.25, 0.5, 0.9, 1.0]
    levels64 = np.linspace(0, 1, 64)
    with partition(cs, k):
        for name, a in _selection_arrays().items():
            t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
            ptr, d = cs.box_of(t)
            p = cs.cube_describe_plan(ptr, d, cs.CUBE_Q_STATS)
            assert p["partition"] == "dynamic", p
            n = int((~np.isnan(a)).sum())
            for r in (0, n // 3, (n - 1) // 2, n - 1):
                assert same_f32(cs.select(t, r), oracle.select(a, r)), (name, k, r)
            m, nv = cs.median(t)
            assert nv == n and m == oracle.median(a), (name, k)
            for lv in (levels, levels64):
                got, nv = cs.quantiles(t, lv)
                want = oracle.quantiles(a, lv)
                assert nv == n
                assert np.array_equal(np.asarray(got).view(np.uint64),
                                      np.asarray(want).view(np.uint64)), (name, k, len(lv))
            if name == "wide":
                assert cs.cube_last_quantile_reads() == 4
            del t


def test_extended_reals_and_offsets_across_chunks(cs):
    """Infinities and NaN payloads in some chunks only, a large offset, and
    blank chunks: the chunk records' merge gives the oracle's reading."""
    rng = np.random.default_rng(5)
    base = rng.standard_normal(300_017).astype(np.float32)
    base[::97] = np.nan
    cases = {}
    a = base.copy(); a[123_457] = np.inf
    cases["plus-inf"] = a
    a = base.copy(); a[200_000] = -np.inf
    cases["minus-inf"] = a
    a = base.copy(); a[5] = np.inf; a[290_000] = -np.inf
    cases["both-inf"] = a
    cases["offset"] = (1e4 + rng.standard_normal(1_000_003) * 1e-3).astype(np.float32)
    a = base.copy(); a[:150_000] = np.nan
    cases["blank-first-half"] = a
    cases["constant"] = np.full(100_000, 3.25, np.float32)
    with partition(cs, 12):
        for name, a in cases.items():
            t = torch.from_numpy(a).cuda()
            ref = oracle.stats(a)
            assert_stats_match(cs.stats(t), ref, name)
            st, c = cs.stats_hist(t, -1.0, 2.0, 64)
            assert_stats_match(st, ref, name + " fused")
            assert_counts_match(c, oracle.hist(a, -1.0, 2.0, 64), name)
