"""The batched persistent launch (GPU) against the oracle and against each
query run alone."""
import numpy as np
import pytest

import oracle
from tests.parity import assert_counts_match, assert_stats_match, same_f32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    return cs


class Outputs:
    """Device output buffers for a list of queries."""

    def __init__(self, n, nbins_max):
        self.out = torch.zeros((n, 64), dtype=torch.uint8, device="cuda")
        self.cnt = torch.zeros((n, nbins_max + 3), dtype=torch.int64, device="cuda")

    def stats(self, cs, i):
        return cs.Stats.from_bytes(self.out[i].cpu().numpy().tobytes())

    def counts(self, i, nbins):
        return self.cnt[i, :nbins + 3].cpu().numpy().view(np.uint64)


def make_items(seed=5, n=12):
    import synth
    rng = np.random.default_rng(seed)
    items = []
    for k in range(n):
        nx, ny, nz = (int(rng.integers(3, 200)), int(rng.integers(1, 60)), int(rng.integers(1, 40)))
        r = synth.WORKLOADS["tiny"].scaled(nx, ny, nz)
        t = synth.cube_tensor(r, 1000 + k, device="cuda")
        items.append(t)
    return items


def queries_for(cs, items, outs, kinds, nbins_list):
    qs = []
    for i, t in enumerate(items):
        ptr, d = cs.box_of(t)
        kind = kinds[i % len(kinds)]
        nb = nbins_list[i % len(nbins_list)]
        lo, hi = -2.5, 20.0
        qs.append(cs.make_query(ptr, d, kind, nb, lo, hi, outs.out[i].data_ptr(),
                                outs.cnt[i].data_ptr()))
    return qs


def check_query(cs, outs, i, t, kind, nb):
    host = t.cpu().numpy()
    ref = oracle.stats(host)
    if kind != cs.CUBE_Q_HIST:
        assert_stats_match(outs.stats(cs, i), ref, f"item {i}")
    if kind in (cs.CUBE_Q_HIST, cs.CUBE_Q_FUSED):
        assert_counts_match(outs.counts(i, nb), oracle.hist(host, -2.5, 20.0, nb), f"item {i}")
    if kind == cs.CUBE_Q_MINMAX:
        assert_counts_match(outs.counts(i, nb), oracle.hist(host, ref.min, ref.max, nb),
                            f"item {i} minmax")


@pytest.mark.parametrize("tile", [4096, 1 << 16, 1 << 20, 0])
def test_mixed_batch_matches_oracle(cs, tile):
    items = make_items()
    kinds = [cs.CUBE_Q_STATS, cs.CUBE_Q_HIST, cs.CUBE_Q_FUSED, cs.CUBE_Q_MINMAX]
    nbins_list = [64, 512, 1000, 7]
    outs = Outputs(len(items), 1000)
    qs = queries_for(cs, items, outs, kinds, nbins_list)
    b = cs.Batch(tile_voxels=tile)
    b.enqueue(qs)
    b.check()
    for i, t in enumerate(items):
        check_query(cs, outs, i, t, kinds[i % 4], nbins_list[i % 4])
    # relaunch and graph replay give the same bits
    ref_out, ref_cnt = outs.out.clone(), outs.cnt.clone()
    for launch in (b.relaunch, b.graph_launch, b.graph_launch, b.graph_launch):
        outs.out.zero_()
        outs.cnt.zero_()
        torch.cuda.synchronize()
        launch()
        b.check()
        assert torch.equal(outs.out, ref_out) and torch.equal(outs.cnt, ref_cnt)
    b.close()


def test_replays_take_their_own_range(cs):
    """Two-pass queries whose cubes change between launches: every relaunch
    and graph replay bins over the new [min, max], never over a range
    published by an earlier launch (the range words carry the launch's
    epoch).  Small tiles give each query many second-phase tiles."""
    items = make_items(seed=9, n=6)
    nb = 64
    outs = Outputs(len(items), nb)
    qs = queries_for(cs, items, outs, [cs.CUBE_Q_MINMAX], [nb])
    b = cs.Batch(tile_voxels=4096)
    b.enqueue(qs)
    b.check()
    for i, t in enumerate(items):
        check_query(cs, outs, i, t, cs.CUBE_Q_MINMAX, nb)
    for k, launch in enumerate((b.graph_launch, b.relaunch, b.graph_launch, b.graph_launch)):
        for t in items:
            t.mul_(1.5).add_(3.0 * (k + 1))   # moves and widens every range
        outs.out.zero_()
        outs.cnt.zero_()
        torch.cuda.synchronize()
        launch()
        b.check()
        for i, t in enumerate(items):
            check_query(cs, outs, i, t, cs.CUBE_Q_MINMAX, nb)
    b.close()


def test_alone_equals_in_mix(cs):
    items = make_items(seed=9, n=10)
    kinds = [cs.CUBE_Q_MINMAX, cs.CUBE_Q_FUSED, cs.CUBE_Q_STATS]
    nbins_list = [512, 256, 1]
    mix = Outputs(len(items), 512)
    b = cs.Batch(tile_voxels=1 << 14)
    b.enqueue(queries_for(cs, items, mix, kinds, nbins_list))
    b.check()
    for i, t in enumerate(items):
        alone = Outputs(1, 512)
        q = queries_for(cs, [t], alone, [kinds[i % 3]], [nbins_list[i % 3]])
        b2 = cs.Batch(tile_voxels=1 << 14)
        b2.enqueue(q)
        b2.check()
        assert torch.equal(alone.out[0], mix.out[i]), f"item {i} stats differ alone vs mix"
        assert torch.equal(alone.cnt[0], mix.cnt[i]), f"item {i} counts differ alone vs mix"
        b2.close()
    b.close()


def test_automatic_tile_sizes(cs):
    """Tile 0: with the default rule each query takes the smallest power of
    two from 2^17 to 2^20 voxels that cuts it into at most 1024 tiles.  Items
    here take 2^17, 2^18 and 2^19; each gives the same bits alone and in the
    mix, and agrees with the oracle."""
    import synth
    shapes = [(37, 11, 5), (200, 300, 9),            # one and five tiles of 2^17
              (1000, 1000, 100),                     # 10^8 voxels: 2^17
              (2048, 1024, 96),                      # 2^27.6 voxels: 2^18
              (2048, 1024, 160)]                     # 2^28.3 voxels: 2^19
    items = [synth.cube_tensor(synth.WORKLOADS["tiny"].scaled(nx, ny, nz), 4200 + k, device="cuda")
             for k, (nx, ny, nz) in enumerate(shapes)]
    kinds = [cs.CUBE_Q_FUSED, cs.CUBE_Q_MINMAX]
    nbins_list = [1024, 333]
    mix = Outputs(len(items), 1024)
    b = cs.Batch(tile_voxels=0)
    b.enqueue(queries_for(cs, items, mix, kinds, nbins_list))
    b.check()
    for i, t in enumerate(items):
        alone = Outputs(1, 1024)
        b2 = cs.Batch(tile_voxels=0)
        b2.enqueue(queries_for(cs, [t], alone, [kinds[i % 2]], [nbins_list[i % 2]]))
        b2.check()
        b2.close()
        assert torch.equal(alone.out[0], mix.out[i]), f"item {i} stats differ alone vs mix"
        assert torch.equal(alone.cnt[0], mix.cnt[i]), f"item {i} counts differ alone vs mix"
        check_query(cs, mix, i, t, kinds[i % 2], nbins_list[i % 2])
    b.close()
    del items
    torch.cuda.empty_cache()


def test_tuned_batch_rule(cs, tmp_path):
    """The batch autotuner picks a rule on a mixed batch; later batches with
    automatic tile and threads run it: every query agrees with the oracle and
    gives the same bits alone and in the mix; the rule survives a save and a
    load of the tuning table."""
    items = make_items(seed=13, n=10)
    kinds = [cs.CUBE_Q_MINMAX, cs.CUBE_Q_FUSED, cs.CUBE_Q_STATS, cs.CUBE_Q_HIST]
    nbins_list = [512, 100, 1, 4096]
    mix = Outputs(len(items), 4096)
    qs = queries_for(cs, items, mix, kinds, nbins_list)
    cs.cube_tune_clear()
    try:
        rep = cs.cube_autotune_batch(qs, reps=2)
        best = rep["best"]
        assert best["threads"] in (256, 512) and rep["candidates"] == 216
        assert best["unroll"] in (2, 4)
        assert 16 <= best["floor_log2"] <= best["cap_log2"] <= 21
        mix.out.zero_()
        mix.cnt.zero_()
        b = cs.Batch(tile_voxels=0, threads=0)
        b.enqueue(qs)
        b.check()
        for i, t in enumerate(items):
            check_query(cs, mix, i, t, kinds[i % 4], nbins_list[i % 4])
            alone = Outputs(1, 4096)
            b2 = cs.Batch(tile_voxels=0, threads=0)
            b2.enqueue(queries_for(cs, [t], alone, [kinds[i % 4]], [nbins_list[i % 4]]))
            b2.check()
            b2.close()
            assert torch.equal(alone.out[0], mix.out[i]), f"item {i} stats differ alone vs mix"
            assert torch.equal(alone.cnt[0], mix.cnt[i]), f"item {i} counts differ alone vs mix"
        b.close()
        path = tmp_path / "t.json"
        cs.cube_tune_save(str(path))
        line = [l for l in open(path) if "batch_threads" in l]
        assert len(line) == 1 and f'"batch_threads": {best["threads"]}' in line[0]
        cs.cube_tune_clear()
        assert cs.cube_tune_load(str(path)) == 1
        cs.cube_tune_save(str(tmp_path / "u.json"))
        assert [l for l in open(tmp_path / "u.json") if "batch_threads" in l] == line
    finally:
        cs.cube_tune_clear()


def test_batch_of_workload_items(cs):
    """The whole 64-item workload (uneven sizes, 1.6e8 voxels), two-pass 512
    bins each, in the form the benchmark times (a graph replay with the
    automatic tile size), every item against the oracle."""
    import synth
    recs = synth.batch_item_recipes()
    items = [synth.cube_tensor(r, synth.BASE_SEED + 2 + i, device="cuda")
             for i, r in enumerate(recs)]
    outs = Outputs(len(items), 512)
    qs = queries_for(cs, items, outs, [cs.CUBE_Q_MINMAX], [512])
    b = cs.Batch(tile_voxels=0)
    b.enqueue(qs)
    b.check()
    first_out, first_cnt = outs.out.clone(), outs.cnt.clone()
    b.graph_launch()
    b.graph_launch()
    b.check()
    b.close()
    assert torch.equal(outs.out, first_out) and torch.equal(outs.cnt, first_cnt)
    for i, t in enumerate(items):
        check_query(cs, outs, i, t, cs.CUBE_Q_MINMAX, 512)
    del items
    torch.cuda.empty_cache()


def test_batch_validation(cs):
    t = torch.zeros(100, device="cuda")
    ptr, d = cs.box_of(t)
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    bad = [cs.make_query(ptr, d, 9, 8, 0, 1, out.data_ptr(), out.data_ptr()),
           cs.make_query(ptr, d, cs.CUBE_Q_HIST, 0, 0, 1, 0, out.data_ptr()),
           cs.make_query(ptr, d, cs.CUBE_Q_HIST, 8, 2, 1, 0, out.data_ptr()),
           cs.make_query(ptr, d, cs.CUBE_Q_STATS, 8, 0, 1, 0, 0),
           cs.make_query(ptr, [1 << 30, 1, 1, 0, 0], cs.CUBE_Q_STATS, 0, 0, 0, out.data_ptr(), 0)]
    for q in bad:
        with pytest.raises(cs.CubeError):
            cs.cube_batch_run([q])
    # an empty box and an empty batch are fine
    cs.cube_batch_run([])
    e = cs.make_query(ptr, [0, 4, 4, 0, 0], cs.CUBE_Q_STATS, 0, 0, 0, out.data_ptr(), 0)
    cs.cube_batch_run([e])
    st = cs.Stats.from_bytes(out.cpu().numpy().tobytes())
    assert st.n_total == 0 and st.flags & cs.CUBE_NO_VALID


def test_query_done_flags_and_order(cs):
    items = make_items(seed=12, n=8)
    outs = Outputs(len(items), 256)
    qs = queries_for(cs, items, outs, [cs.CUBE_Q_MINMAX, cs.CUBE_Q_STATS], [256])
    b = cs.Batch(tile_voxels=1 << 14)
    b.set_order(cs.CUBE_ORDER_SMALLEST_FIRST)
    b.enqueue(qs)
    b.check()
    assert all(b.query_done(i) for i in range(len(items)))
    for i, t in enumerate(items):
        check_query(cs, outs, i, t, [cs.CUBE_Q_MINMAX, cs.CUBE_Q_STATS][i % 2], 256)
    b.relaunch()
    b.check()
    assert all(b.query_done(i) for i in range(len(items)))
    assert not b.query_done(len(items) + 1000)
    with pytest.raises(cs.CubeError):
        b.set_order(7)
    b.close()


def test_relaunch_across_streams_is_ordered(cs):
    """Launches of one batch on different streams run one after another
    (they share the batch's device state): every launch's outputs equal the
    first launch's, with no host synchronisation between the launches."""
    items = make_items(seed=21, n=10)
    outs = Outputs(len(items), 512)
    kinds = [cs.CUBE_Q_MINMAX, cs.CUBE_Q_FUSED, cs.CUBE_Q_STATS, cs.CUBE_Q_HIST]
    qs = queries_for(cs, items, outs, kinds, [512, 64])
    b = cs.Batch(tile_voxels=1 << 12)
    s = [torch.cuda.Stream() for _ in range(3)]
    b.enqueue(qs, s[0].cuda_stream)
    b.check()
    first_out, first_cnt = outs.out.clone(), outs.cnt.clone()
    for rep in range(4):
        outs.out.zero_()
        outs.cnt.zero_()
        torch.cuda.synchronize()
        b.relaunch(s[1].cuda_stream)
        b.graph_launch(s[2].cuda_stream)
        b.relaunch(s[0].cuda_stream)
        b.graph_launch(s[1].cuda_stream)
        b.check()
        torch.cuda.synchronize()
        assert torch.equal(outs.out, first_out), rep
        assert torch.equal(outs.cnt, first_cnt), rep
    b.close()
    for i, t in enumerate(items):
        check_query(cs, outs, i, t, kinds[i % len(kinds)], [512, 64][i % 2])


def test_batch64_workload_precision(cs):
    """The 64-cube batch workload: every item's batched result (FP64 merge of
    compensated FP32 partials) against the oracle, and the same items through
    the naive-FP32 and Kahan-FP32 modes of the single-box pass, whose errors
    are reported beside it.  Only the production path is held to 1e-6."""
    import synth
    recs = synth.batch_item_recipes()
    items = [synth.cube_tensor(r, synth.BASE_SEED + 2 + i, device="cuda")
             for i, r in enumerate(recs)]
    nb = synth.HIST_BINS["batch64"]
    outs = Outputs(len(items), nb)
    qs = [cs.make_query(*cs.box_of(t), cs.CUBE_Q_MINMAX, nb, 0.0, 0.0, outs.out[i].data_ptr(),
                        outs.cnt[i].data_ptr()) for i, t in enumerate(items)]
    b = cs.Batch(tile_voxels=1 << 18)
    b.enqueue(qs)
    b.check()
    b.close()
    worst = {"batched": 0.0, "naive32": 0.0, "kahan32": 0.0}
    try:
        for i, t in enumerate(items):
            host = t.cpu().numpy()
            ref = oracle.stats(host)
            st = outs.stats(cs, i)
            assert_stats_match(st, ref, f"batched item {i}")
            assert_counts_match(outs.counts(i, nb), oracle.hist(host, ref.min, ref.max, nb),
                                f"batched item {i}")
            worst["batched"] = max(worst["batched"], abs(st.std - ref.std) / ref.std)
            for mode, name in ((cs.CUBE_ACCUM_NAIVE32, "naive32"),
                               (cs.CUBE_ACCUM_KAHAN32, "kahan32")):
                cs.cube_set_accum_mode(mode)
                s2 = cs.stats(t)
                assert s2.n_valid == ref.n_valid and same_f32(s2.max, ref.max)
                worst[name] = max(worst[name], abs(s2.std - ref.std) / ref.std)
            cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    finally:
        cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    print("batch64 worst std rel err:", worst)
    assert worst["batched"] <= 1e-6


def test_expired_range_wait_fails_only_its_query(cs, monkeypatch):
    """A two-pass query whose bounded wait for its own range gives up (forced
    from the host: in launch 1 of this batch every range wait gives up at
    once, and every kernel still runs to its end) completes marked as failed;
    the other queries of the batch are unaffected; the batch's check reports
    it once.  The next launch -- over data changed in place, so a range left
    up by launch 1 would give wrong bins -- is whole and correct again."""
    monkeypatch.setenv("CUBE_FAULT_INJECT", "expire:1")
    b = cs.Batch(tile_voxels=1 << 14)
    monkeypatch.delenv("CUBE_FAULT_INJECT")
    items = make_items(seed=17, n=8)
    kinds = [cs.CUBE_Q_MINMAX, cs.CUBE_Q_STATS, cs.CUBE_Q_FUSED, cs.CUBE_Q_HIST]
    outs = Outputs(len(items), 256)
    qs = queries_for(cs, items, outs, kinds, [256, 64])
    b.enqueue(qs)
    torch.cuda.synchronize()
    for i in range(len(items)):
        kind = kinds[i % len(kinds)]
        if kind == cs.CUBE_Q_MINMAX:
            with pytest.raises(cs.CubeError, match="expired"):
                b.query_done(i)
        else:
            assert b.query_done(i)
            check_query(cs, outs, i, items[i], kind, [256, 64][i % 2])
    with pytest.raises(cs.CubeError, match="timed out"):
        b.check()
    b.check()                      # reported once
    for t in items:                # new data under the same pointers
        t.mul_(-3.0).add_(7.0)
    outs.cnt.zero_()
    b.relaunch()
    b.check()
    for i in range(len(items)):
        assert b.query_done(i)
        check_query(cs, outs, i, items[i], kinds[i % len(kinds)], [256, 64][i % 2])
    b.close()
