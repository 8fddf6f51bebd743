"""The query server (GPU): results in a concurrent mix equal the same query
alone, and the plain mode agrees with the batched mode."""
import threading
import time

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
    return cs


@pytest.fixture(scope="module")
def cubes():
    import synth
    rs = synth.serve_recipes(scale_div=16)[:6]
    return [synth.cube_tensor(r, 300 + i, device="cuda") for i, r in enumerate(rs)]


def random_queries(cs, cubes, n, seed, nbins_max=1024):
    """(query, cube index, box slices, kind, nbins, lo, hi) of a random mix."""
    rng = np.random.default_rng(seed)
    out = torch.zeros((n, 64), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros((n, nbins_max + 3), dtype=torch.int64, device="cuda")
    specs = []
    for i in range(n):
        c = int(rng.integers(len(cubes)))
        t = cubes[c]
        nz, ny, nx = t.shape
        if rng.random() < 0.4:
            sl = np.s_[:, :, :]
        else:
            z0, y0, x0 = (int(rng.integers(0, max(1, s // 2))) for s in (nz, ny, nx))
            z1 = int(rng.integers(z0 + 1, nz + 1))
            y1 = int(rng.integers(y0 + 1, ny + 1))
            x1 = int(rng.integers(x0 + 1, nx + 1))
            sl = np.s_[z0:z1, y0:y1, x0:x1]
        kind = int(rng.choice([cs.CUBE_Q_STATS, cs.CUBE_Q_HIST, cs.CUBE_Q_FUSED, cs.CUBE_Q_MINMAX]))
        nb = int(rng.choice([64, 256, 1024]))
        lo, hi = float(rng.uniform(-4, -1)), float(rng.uniform(1, 30))
        ptr, d = cs.box_of(t[sl])
        q = cs.make_query(ptr, d, kind, nb, lo, hi, out[i].data_ptr(), cnt[i].data_ptr())
        specs.append((q, c, sl, kind, nb, lo, hi))
    return specs, out, cnt


@pytest.mark.parametrize("tile", [1 << 16, 0])
def test_server_mix_equals_alone(cs, cubes, tile):
    """tile 0: each query's automatic tile size (the server's default)."""
    specs, out, cnt = random_queries(cs, cubes, 60, seed=3)
    srv = cs.Server(cs.CUBE_SERVE_BATCHED, slots=3, max_batch=8, tile_voxels=tile)
    # submit from two threads with staggered arrivals
    ids = [None] * len(specs)

    def submitter(part):
        for i in part:
            ids[i] = srv.submit(specs[i][0])
            time.sleep(0.0005)

    th = [threading.Thread(target=submitter, args=(range(k, len(specs), 2),)) for k in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    lat = [srv.wait(i, timeout_s=60) for i in ids]
    assert all(x >= 0 for x in lat)
    p50, p99, n = srv.latency()
    assert n == len(specs) and p99 >= p50 > 0
    srv.close()
    torch.cuda.synchronize()
    # each query alone through its own batch gives the same bits
    for i, (q, c, sl, kind, nb, lo, hi) in enumerate(specs):
        o1 = torch.zeros(64, dtype=torch.uint8, device="cuda")
        c1 = torch.zeros(nb + 3, dtype=torch.int64, device="cuda")
        q1 = cs.make_query(q.ptr, list(q.dims), kind, nb, lo, hi, o1.data_ptr(), c1.data_ptr())
        b = cs.Batch(tile_voxels=tile)
        b.enqueue([q1])
        b.check()
        b.close()
        if kind != cs.CUBE_Q_HIST:
            assert torch.equal(o1, out[i]), f"query {i} stats differ alone vs in the mix"
        if kind != cs.CUBE_Q_STATS:
            assert torch.equal(c1, cnt[i, :nb + 3]), f"query {i} counts differ"
    # and every served query agrees with the oracle
    hosts = [t.cpu().numpy() for t in cubes]
    for i in range(len(specs)):
        q, c, sl, kind, nb, lo, hi = specs[i]
        host = hosts[c][sl]
        ref = oracle.stats(host)
        if kind != cs.CUBE_Q_HIST:
            st = cs.Stats.from_bytes(out[i].cpu().numpy().tobytes())
            assert_stats_match(st, ref, f"query {i}")
        got = cnt[i, :nb + 3].cpu().numpy().view(np.uint64)
        if kind in (cs.CUBE_Q_HIST, cs.CUBE_Q_FUSED):
            assert_counts_match(got, oracle.hist(host, lo, hi, nb), f"query {i}")
        elif kind == cs.CUBE_Q_MINMAX and ref.n_valid:
            assert_counts_match(got, oracle.hist(host, ref.min, ref.max, nb), f"query {i}")


def test_plain_mode_agrees(cs, cubes):
    specs, out, cnt = random_queries(cs, cubes, 20, seed=4)
    srv = cs.Server(cs.CUBE_SERVE_PLAIN)
    ids = [srv.submit(s[0]) for s in specs]
    for i in ids:
        srv.wait(i, timeout_s=60)
    srv.close()
    for i, (q, c, sl, kind, nb, lo, hi) in enumerate(specs):
        host = cubes[c].cpu().numpy()[sl]
        ref = oracle.stats(host)
        if kind != cs.CUBE_Q_HIST:
            assert_stats_match(cs.Stats.from_bytes(out[i].cpu().numpy().tobytes()), ref, f"q{i}")
        got = cnt[i, :nb + 3].cpu().numpy().view(np.uint64)
        if kind in (cs.CUBE_Q_HIST, cs.CUBE_Q_FUSED):
            assert_counts_match(got, oracle.hist(host, lo, hi, nb), f"q{i}")


def test_server_rejects_bad_queries(cs, cubes):
    srv = cs.Server()
    t = cubes[0]
    ptr, d = cs.box_of(t)
    o = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(cs.CubeError):
        srv.submit(cs.make_query(ptr, d, 7, 8, 0, 1, o.data_ptr(), o.data_ptr()))
    with pytest.raises(cs.CubeError):
        srv.submit(cs.make_query(ptr, d, cs.CUBE_Q_HIST, 8, 1, 0, 0, o.data_ptr()))
    with pytest.raises(cs.CubeError):
        srv.wait(12345, timeout_s=0.01)
    srv.close()


def test_early_completions_counted_once(cs):
    """Small queries finish (by their completion flags) and are collected by
    wait() long before the large query of the same batch: each latency is
    recorded once, and collected ids are never brought back."""
    big = torch.randn(1 << 28, device="cuda")
    small = [torch.randn(4096, device="cuda") for _ in range(7)]
    out = torch.zeros((8, 64), dtype=torch.uint8, device="cuda")
    srv = cs.Server(cs.CUBE_SERVE_BATCHED, slots=1, max_batch=8, tile_voxels=1 << 16)
    for rep in range(3):
        qs = [cs.make_query(*cs.box_of(t), cs.CUBE_Q_STATS, 0, 0.0, 0.0, out[i].data_ptr())
              for i, t in enumerate([big] + small)]
        ids = [srv.submit(q) for q in qs]
        for i in ids[1:] + ids[:1]:      # the small ones first
            assert srv.wait(i, timeout_s=60) >= 0
        time.sleep(0.05)                 # let the worker see the batch's event
        p50, p99, n = srv.latency(reset=True)
        assert n == len(qs), (rep, n)
    srv.close()
    torch.cuda.synchronize()
    for i, t in enumerate(small):
        st = cs.Stats.from_bytes(out[i + 1].cpu().numpy().tobytes())
        assert st.n_valid == 4096 and st.max == float(t.max())


def test_injected_launch_failure_is_isolated(cs, monkeypatch):
    """A launch that fails (forced on the host: launches 2 and 4 of this
    server) fails exactly the queries of that batch, with the error reported
    to their waiters; the server goes on serving the rest correctly."""
    monkeypatch.setenv("CUBE_FAULT_INJECT", "launch:2,4")
    t = torch.randn(1 << 16, device="cuda")
    ref = oracle.stats(t.cpu().numpy())
    out = torch.zeros((6, 64), dtype=torch.uint8, device="cuda")
    srv = cs.Server(cs.CUBE_SERVE_BATCHED, slots=1, max_batch=1)
    monkeypatch.delenv("CUBE_FAULT_INJECT")
    results = []
    for i in range(6):     # one query per batch: submit, then wait
        qid = srv.submit(cs.make_query(*cs.box_of(t), cs.CUBE_Q_STATS, 0, 0.0, 0.0,
                                       out[i].data_ptr()))
        try:
            srv.wait(qid, timeout_s=60)
            results.append("ok")
        except cs.CubeError as e:
            assert "injected" in str(e)
            results.append("failed")
    assert results == ["ok", "failed", "ok", "failed", "ok", "ok"]
    _, _, n = srv.latency()
    assert n == 4
    srv.close()
    torch.cuda.synchronize()
    for i in (0, 2, 4, 5):
        assert_stats_match(cs.Stats.from_bytes(out[i].cpu().numpy().tobytes()), ref, f"query {i}")


def test_injected_event_error_is_isolated(cs, monkeypatch):
    """A launch whose completion event reports a device error (forced from
    the host for launch 2: the work itself runs to its end) fails the
    queries of that launch with the error; the slot is freed, the server
    goes on serving, and destroying it returns."""
    monkeypatch.setenv("CUBE_FAULT_INJECT", "event:2")
    t = torch.randn(1 << 16, device="cuda")
    ref = oracle.stats(t.cpu().numpy())
    out = torch.zeros((5, 64), dtype=torch.uint8, device="cuda")
    for mode in (cs.CUBE_SERVE_BATCHED, cs.CUBE_SERVE_PLAIN):
        out.zero_()
        srv = cs.Server(mode, slots=1, max_batch=1)
        results = []
        for i in range(5):
            qid = srv.submit(cs.make_query(*cs.box_of(t), cs.CUBE_Q_STATS, 0, 0.0, 0.0,
                                           out[i].data_ptr()))
            try:
                srv.wait(qid, timeout_s=60)
                results.append("ok")
            except cs.CubeError as e:
                assert "failed on the device" in str(e)
                results.append("failed")
        assert results == ["ok", "failed", "ok", "ok", "ok"], (mode, results)
        _, _, n = srv.latency()
        assert n == 4
        srv.close()
        torch.cuda.synchronize()
        for i in (0, 2, 3, 4):
            assert_stats_match(cs.Stats.from_bytes(out[i].cpu().numpy().tobytes()), ref, f"q{i}")
    monkeypatch.delenv("CUBE_FAULT_INJECT")


def test_expired_range_wait_fails_only_its_query_served(cs, cubes, monkeypatch):
    """In the first launch of each slot every range wait gives up at once
    (forced from the host; every kernel still ends normally): exactly the
    two-pass queries of those launches fail, every other query is served
    correctly, later launches of the same slots are whole, and destroying
    the server returns."""
    monkeypatch.setenv("CUBE_FAULT_INJECT", "expire:1")
    srv = cs.Server(cs.CUBE_SERVE_BATCHED, slots=2, max_batch=6)
    monkeypatch.delenv("CUBE_FAULT_INJECT")
    specs, out, cnt = random_queries(cs, cubes, 24, seed=9, nbins_max=1024)
    # the first query opens the first launch: make it a two-pass one
    q, c, sl, kind, nb, lo, hi = specs[0]
    q.kind = cs.CUBE_Q_MINMAX
    specs[0] = (q, c, sl, cs.CUBE_Q_MINMAX, nb, lo, hi)
    ids = [srv.submit(s[0]) for s in specs]
    failed = set()
    for i, qid in enumerate(ids):
        try:
            srv.wait(qid, timeout_s=60)
        except cs.CubeError as e:
            assert "expired" in str(e), str(e)
            failed.add(i)
    srv.close()
    torch.cuda.synchronize()
    assert 0 in failed
    assert all(specs[i][3] == cs.CUBE_Q_MINMAX for i in failed)
    hosts = [t.cpu().numpy() for t in cubes]
    for i, (q, c, sl, kind, nb, lo, hi) in enumerate(specs):
        if i in failed:
            continue
        host = hosts[c][sl]
        ref = oracle.stats(host)
        if kind != cs.CUBE_Q_HIST:
            assert_stats_match(cs.Stats.from_bytes(out[i].cpu().numpy().tobytes()), ref, f"q{i}")
        got = cnt[i, :nb + 3].cpu().numpy().view(np.uint64)
        if kind in (cs.CUBE_Q_HIST, cs.CUBE_Q_FUSED):
            assert_counts_match(got, oracle.hist(host, lo, hi, nb), f"q{i}")
        elif kind == cs.CUBE_Q_MINMAX and ref.n_valid:
            assert_counts_match(got, oracle.hist(host, ref.min, ref.max, nb), f"q{i}")
