"""Full-size parity (GPU, slow): the 16 GiB brick against the oracle over the
whole cube, in the launch configuration the benchmark times; the
precision-stress recipe (offset 1e4, noise 1e-3, sources up to 1e3) at 16 GiB,
where the FP32-only accumulation modes are reported beside the production
FP64-merge path; the full 128 GiB stress cube, by properties, sampled
sub-boxes and ranks; and the serving set at its real size (about 201 GiB).

The oracle runs on host copies (the 128 GiB cube slab by slab on host
threads); these tests take a minute or two each and are marked `slow` as well
as `gpu`.
"""
import os
import time

import numpy as np
import pytest

import oracle
from tests.devstream import host_threads, oracle_stats_of_device
from tests.parity import assert_counts_match, assert_stats_match, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    """The library in the launch configuration bench.py times: the shipped
    gfx950 tuning table loaded, no explicit shape."""
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    table = os.path.join(os.path.dirname(cs.__file__), "tuning", "gfx950.json")
    assert cs.cube_tune_load(table) >= 1
    yield cs
    cs.cube_tune_clear()


def _host_copy(t):
    h = np.empty(tuple(t.shape), dtype=np.float32)
    step = 64
    for z in range(0, t.shape[0], step):
        h[z:z + step] = t[z:z + step].cpu().numpy()
    return h


@pytest.mark.timeout(600)
def test_brick16g_full_cube(cs):
    import synth
    name = "brick16g"
    r = synth.WORKLOADS[name]
    nb = synth.HIST_BINS[name]
    t = synth.cube_tensor(r, synth.BASE_SEED + 1, device="cuda")
    # the shipped table's plan for this box: the dynamic partition bench.py times
    ptr, d = cs.box_of(t)
    plan = cs.cube_describe_plan(ptr, d, cs.CUBE_Q_FUSED, nb)
    print("brick16g fused plan:", plan)
    assert plan["partition"] == "dynamic" and plan["chunks"] == r.n >> 18, plan
    st_fused_ref = cs.stats(t)
    st, counts = cs.stats_hist(t, st_fused_ref.min, st_fused_ref.max, nb)
    st2, counts2 = cs.stats_hist_minmax(t, nb)
    k_mid = (int(st_fused_ref.n_valid) - 1) // 2
    sel = {k: cs.select(t, k) for k in (0, k_mid, int(st_fused_ref.n_valid) - 1)}
    med, med_nv = cs.median(t)
    probe = cs.read_probe(t, nb)
    # quantiles at two levels whose ranks need interpolation, and the voxels
    # of the two ranks around each
    qlv = [0.25, 0.9]
    qv, qn = cs.quantiles(t, qlv)
    qpairs = []
    for lvl in qlv:
        h = lvl * (qn - 1)
        j = int(np.floor(h))
        qpairs.append((j, h - j, cs.select(t, j), cs.select(t, j + 1)))
    t0 = time.perf_counter()
    host = _host_copy(t)
    del t
    torch.cuda.empty_cache()
    ref = oracle.stats(host)
    want = oracle.hist(host, ref.min, ref.max, nb)
    print(f"oracle over 2^32 voxels: {time.perf_counter() - t0:.1f} s")
    for got, what in ((st, "fused"), (st2, "two-pass"), (st_fused_ref, "stats")):
        assert_stats_match(got, ref, what)
        print(what, "rel err (mean, std):", rel_err(got, ref))
    assert_counts_match(counts, want, "fused counts")
    assert_counts_match(counts2, want, "two-pass counts")
    assert int(want.sum()) == r.n
    # quantiles: the interpolation (the oracle's, over the two voxels) of
    # the voxels of ranks j and j + 1, each checked by counting
    assert qn == ref.n_valid
    for (j, f, a, b), got in zip(qpairs, qv):
        assert got == oracle.quantiles(np.array([a, b], np.float32), [f])[0]
        for rank, v in ((j, a), (j + 1, b)):
            assert int(np.count_nonzero(host < v)) <= rank < int(np.count_nonzero(host <= v))
    # the read probe saw every voxel's bits
    assert probe == int(np.bitwise_or.reduce(host.view(np.uint32).reshape(-1)))
    # Selection at full size, by the rank property that fixes the k-th
    # smallest: at most k valid voxels lie below it and more than k at or
    # below it (so it is one of the voxels).  The extremes are the min/max.
    assert sel[0] == ref.min and sel[int(ref.n_valid) - 1] == ref.max
    v = sel[k_mid]
    below = int(np.count_nonzero(host < v))
    at_or_below = int(np.count_nonzero(host <= v))
    assert below <= k_mid < at_or_below, (v, below, at_or_below, k_mid)
    assert med_nv == ref.n_valid
    if ref.n_valid % 2:
        assert med == v
    else:
        upper = float(np.min(host[host > v])) if at_or_below == k_mid + 1 else v
        assert med == (float(v) + upper) / 2.0


@pytest.mark.timeout(600)
def test_precision_stress_16g(cs):
    import synth
    base = synth.WORKLOADS["stress128g"]
    r = base.scaled(2048, 2048, 1024)
    t = synth.cube_tensor(r, synth.BASE_SEED + 4, device="cuda")
    errs = {}
    got = {}
    try:
        for mode, name in ((cs.CUBE_ACCUM_NAIVE32, "naive32"), (cs.CUBE_ACCUM_KAHAN32, "kahan32"),
                           (cs.CUBE_ACCUM_FP64MERGE, "fp64merge")):
            cs.cube_set_accum_mode(mode)
            got[name] = cs.stats(t)
    finally:
        cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    host = _host_copy(t)
    del t
    torch.cuda.empty_cache()
    ref = oracle.stats(host)
    for name, st in got.items():
        errs[name] = rel_err(st, ref)
        assert st.n_valid == ref.n_valid and st.min == ref.min and st.max == ref.max
    print("precision stress (mean err, std err):", errs)
    assert_stats_match(got["fp64merge"], ref, "fp64merge")
    assert errs["naive32"][1] > errs["fp64merge"][1]
    out = os.environ.get("CUBE_PRECISION_REPORT")
    if out:
        import json
        with open(out, "w") as f:
            json.dump({"recipe": "stress128g scaled to 2048x2048x1024", "oracle_std": ref.std,
                       "oracle_mean": ref.mean,
                       "rel_err_mean_std": {k: list(v) for k, v in errs.items()}}, f, indent=1)


@pytest.mark.timeout(900)
def test_stress128g_full_size(cs):
    """The 128 GiB stress cube (2^35 voxels) in the launch configuration the
    benchmark times: properties that hold at any size on the whole cube; the
    whole cube's statistics against the oracle (streamed to host threads),
    for the stats, fused and two-pass calls, with the oracle-relative errors
    of the three accumulation modes; sub-boxes at the start, the middle and
    the far end (element offsets past 2^34) against the oracle; and
    selection, median and quantiles checked by their ranks (counted on the
    GPU, a chunk of planes at a time)."""
    import synth
    r = synth.WORKLOADS["stress128g"]
    nb = synth.HIST_BINS["stress128g"]
    t = synth.cube_tensor(r, synth.BASE_SEED + 4, device="cuda")
    nz = t.shape[0]
    st = cs.stats(t)
    assert st.n_total == r.n and st.n_valid + st.n_nan == r.n
    st_f, c_f = cs.stats_hist(t, st.min, st.max, nb)
    st_2, c_2 = cs.stats_hist_minmax(t, nb)
    assert np.array_equal(c_f, c_2)
    assert int(c_f.sum()) == r.n and int(c_f[nb]) == 0 and int(c_f[nb + 1]) == 0
    assert int(c_f[nb + 2]) == st.n_nan
    for s in (st_f, st_2):
        assert s.min == st.min and s.max == st.max and s.n_valid == st.n_valid
        assert abs(s.mean - st.mean) <= 1e-9 * abs(st.mean) and abs(s.std - st.std) <= 1e-6 * st.std

    # the whole cube against the oracle (streamed slab by slab to host
    # threads): the production path under the tolerance rule, and the
    # FP32-only modes reported beside it, relative to the oracle
    t0 = time.perf_counter()
    ref = oracle_stats_of_device(oracle, t)
    t_oracle = time.perf_counter() - t0
    assert_stats_match(st, ref, "stats, whole stress cube")
    assert_stats_match(st_f, ref, "fused, whole stress cube")
    assert_stats_match(st_2, ref, "two-pass, whole stress cube")
    modes = {}
    try:
        for mode, name in ((cs.CUBE_ACCUM_NAIVE32, "naive32"), (cs.CUBE_ACCUM_KAHAN32, "kahan32"),
                           (cs.CUBE_ACCUM_FP64MERGE, "fp64merge")):
            cs.cube_set_accum_mode(mode)
            modes[name] = rel_err(cs.stats(t), ref)
    finally:
        cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    print(f"stress128g whole cube vs oracle ({t_oracle:.0f} s of oracle on "
          f"{host_threads()} threads), (mean err, std err): {modes}")
    assert modes["fp64merge"][0] <= 1e-6 and modes["fp64merge"][1] <= 1e-6
    assert modes["naive32"][1] > modes["fp64merge"][1]
    out = os.environ.get("CUBE_PRECISION_REPORT")
    if out:
        import json
        with open(out, "w") as f:
            json.dump({"recipe": "stress128g, 4096x4096x2048 (2^35 voxels)",
                       "oracle_mean": ref.mean, "oracle_std": ref.std,
                       "oracle_seconds": t_oracle, "threads": host_threads(),
                       "rel_err_mean_std": {k: list(v) for k, v in modes.items()}}, f, indent=1)
    golden = os.path.join(os.path.dirname(__file__), "golden", "stress128g_oracle.json")
    if os.path.exists(golden):
        import dataclasses
        import json
        from tests.golden.make_stress128g_oracle import generator_hash
        g = json.load(open(golden))
        if g["generator_sha256_16"] == generator_hash() and g["seed"] == synth.BASE_SEED + 4:
            # the stored oracle values are those of this cube, bit for bit
            assert g["stats"] == dataclasses.asdict(ref), (g["stats"], ref)

    # sub-boxes against the oracle, including the far end of the cube
    for sl in (np.s_[0:2], np.s_[nz // 2:nz // 2 + 2, 100:3000, 7:4001], np.s_[nz - 2:nz]):
        sub = t[sl]
        host = sub.cpu().numpy()
        ref = oracle.stats(host)
        assert_stats_match(cs.stats(sub), ref, f"stats {sl}")
        if ref.n_valid:
            s2, c2 = cs.stats_hist_minmax(sub, nb)
            assert_stats_match(s2, ref, f"two-pass {sl}")
            assert_counts_match(c2, oracle.hist(host, ref.min, ref.max, nb), f"counts {sl}")
        del sub, host

    def count_below(v, inclusive):
        n = 0
        for z0 in range(0, nz, 128):
            blk = t[z0:z0 + 128]
            n += int(((blk <= v) if inclusive else (blk < v)).sum())
        return n

    def rank_holds(v, k):
        return count_below(v, False) <= k < count_below(v, True)

    n = int(st.n_valid)
    k_mid = (n - 1) // 2
    v = cs.select(t, k_mid)
    assert rank_holds(v, k_mid)
    med, med_n = cs.median(t)
    assert med_n == n
    if n % 2 == 0:
        nxt = cs.select(t, k_mid + 1)
        assert med == (float(v) + float(nxt)) / 2.0
    else:
        assert med == v
    qv, qn = cs.quantiles(t, [0.0, 0.25, 0.75, 1.0])
    assert qn == n and qv[0] == st.min and qv[3] == st.max
    for lvl, got in ((0.25, qv[1]), (0.75, qv[2])):
        h = lvl * (n - 1)
        j = int(np.floor(h))
        a, b = cs.select(t, j), cs.select(t, j + 1)
        assert got == oracle.quantiles(np.array([a, b], np.float32), [h - j])[0]
        assert rank_holds(a, j) and rank_holds(b, j + 1)
    del t
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_serving_full_size(cs):
    """The serving workload at its real size: twelve resident cubes (about
    201 GiB, the largest 2^34 voxels) and the seeded query mix, plus
    minmax-histogram queries.  Every served result equals the single-box
    calls bit for bit (same tiling-independent counts and extrema, same
    statistics bytes when the single-box pass is run as a one-query batch);
    the 50 smallest served queries are checked against the oracle."""
    import threading

    import synth
    from paper_1111_6661_amd import workloads
    recipes = synth.serve_recipes()
    cubes = [synth.cube_tensor(r, synth.BASE_SEED + 3 + i, device="cuda")
             for i, r in enumerate(recipes)]
    try:
        ranges = []
        for c in cubes:
            s = cs.stats(c)
            ranges.append(((s.min, s.max), (s.mean - 2 * s.std, s.mean + 2 * s.std)))
        shapes = [tuple(c.shape) for c in cubes]
        specs = workloads.query_stream(shapes, ranges, 80, 1e9, synth.BASE_SEED + 40,
                                       cs.CUBE_Q_STATS, cs.CUBE_Q_FUSED)
        n = len(specs)
        out = torch.zeros((n, 64), dtype=torch.uint8, device="cuda")
        cnt = torch.zeros((n, 4096 + 3), dtype=torch.int64, device="cuda")
        qs, views = [], []
        for i, q in enumerate(specs):
            z0, z1, y0, y1, x0, x1 = q.box
            v = cubes[q.cube][z0:z1, y0:y1, x0:x1]
            kind = q.kind if i % 5 else cs.CUBE_Q_MINMAX
            nb = q.nbins or 256
            p, d = cs.box_of(v)
            qs.append(cs.make_query(p, d, kind, nb, q.lo, q.hi, out[i].data_ptr(),
                                    cnt[i].data_ptr()))
            views.append((v, kind, nb, q.lo, q.hi))
        srv = cs.Server(cs.CUBE_SERVE_BATCHED, slots=4, max_batch=32)
        ids = [0] * n

        def submit():
            for i, q in enumerate(qs):
                ids[i] = srv.submit(q)

        th = threading.Thread(target=submit)
        th.start()
        th.join()
        for i in ids:
            assert srv.wait(i, timeout_s=120) >= 0
        srv.close()
        torch.cuda.synchronize()
        for i, (v, kind, nb, lo, hi) in enumerate(views):
            # the same query alone, through a one-query batch with the
            # server's automatic tile: identical bytes
            o1 = torch.zeros(64, dtype=torch.uint8, device="cuda")
            c1 = torch.zeros(nb + 3, dtype=torch.int64, device="cuda")
            p, d = cs.box_of(v)
            b = cs.Batch(tile_voxels=0)
            b.enqueue([cs.make_query(p, d, kind, nb, lo, hi, o1.data_ptr(), c1.data_ptr())])
            b.check()
            b.close()
            assert torch.equal(o1, out[i]), f"query {i} stats differ from the query alone"
            if kind != cs.CUBE_Q_STATS:
                assert torch.equal(c1, cnt[i, :nb + 3]), f"query {i} counts differ"
            # and the plain single-box calls: exact counts and extrema
            st = cs.Stats.from_bytes(out[i].cpu().numpy().tobytes())
            ref = cs.stats(v)
            assert st.n_valid == ref.n_valid and st.n_nan == ref.n_nan
            assert same_bits(st.min, ref.min) and same_bits(st.max, ref.max)
            if kind == cs.CUBE_Q_FUSED:
                _, cf = cs.stats_hist(v, lo, hi, nb)
                assert np.array_equal(cnt[i, :nb + 3].cpu().numpy().view(np.uint64), cf)
            elif kind == cs.CUBE_Q_MINMAX:
                _, cm = cs.stats_hist_minmax(v, nb)
                assert np.array_equal(cnt[i, :nb + 3].cpu().numpy().view(np.uint64), cm)
        # the 50 smallest served queries against the oracle (statistics of
        # every one, streamed to host threads; counts of those up to 2^27
        # voxels)
        small = sorted(range(n), key=lambda i: specs[i].voxels)[:50]
        for i in small:
            v, kind, nb, lo, hi = views[i]
            ref = oracle_stats_of_device(oracle, v)
            if kind != cs.CUBE_Q_HIST:
                assert_stats_match(cs.Stats.from_bytes(out[i].cpu().numpy().tobytes()), ref,
                                   f"served query {i}")
            if kind != cs.CUBE_Q_STATS and v.numel() <= (1 << 27):
                host = v.cpu().numpy()
                want = oracle.hist(host, lo, hi, nb) if kind != cs.CUBE_Q_MINMAX else \
                    oracle.hist(host, ref.min, ref.max, nb) if ref.n_valid else None
                if want is not None:
                    assert_counts_match(cnt[i, :nb + 3].cpu().numpy().view(np.uint64), want,
                                        f"served query {i} counts")
    finally:
        del cubes
        torch.cuda.empty_cache()


def same_bits(a, b):
    return np.float32(a).view(np.uint32) == np.float32(b).view(np.uint32)
