#!/usr/bin/env python3
"""Benchmark: fused statistics + histogram pass over one GPU's 16 GiB brick.

A step is one fused launch (cube_stats_hist_async) over a resident float32
cube of 2048 x 2048 x 1024 voxels (16 GiB; noise + 10^4 Gaussian sources with
peak amplitude log-uniform in [3, 1000] + 1 % blank voxels in channel ranges
and whole pixels), with a 1024-bin histogram over the cube's [min, max]:
min, max, blank count, mean, std and the histogram in one read of HBM.

The JSON line carries:
  value       voxels per second of the fused pass (inputs resident in HBM);
  roofline    the fused kernel's algorithmic bytes (4 per voxel) per launch
              divided by its average launch duration, measured with HIP events
              on the launch stream, against the 8 TB/s HBM peak, with the read
              ceiling of the same access pattern (the read probe) beside it;
  cpu_baseline the oracle (single thread) on a bounded sample of the cube;
  p50_ms/p99_ms query latency of the continuous-batching server replaying a
              seeded Poisson query mix over 12 resident cubes (about 201 GiB);
  extra       the read probe; two-pass [min, max], stats-only and
              histogram-only timings; the 64-cube batch (graph replay vs plain
              launches, tile sizes including the automatic one); selection,
              median and quantiles; projection maps; out-of-core queries from
              host memory; the 128 GiB precision-stress cube; the serving
              replay (plain vs served, and served with one fixed tile size);
              the launch shapes used; parity checks of each.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       [--tune table|run|off] [--tune-save PATH] [--only-fused] [--no-...]
       [--serve-seconds S] [--serve-sweep 0.5,0.9]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MIN_SERVE_QUERIES = 10_000


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_launches(fn, stream, steps: int, warmup: int):
    """Run fn() warmup + steps times on `stream`; return (wall ms per step,
    mean event ms per launch)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = [a.elapsed_time(b) for a, b in evs]
    time_launches.last = per          # per-launch event times of the last call
    return wall, sum(per) / steps


def prewarm(fn, stream, ms: float) -> int:
    """Run fn() back to back for about `ms` of wall time, untimed; return the
    launches.  After the GPU idles its shader clock falls, and the fused pass
    (about 80 % VALU-busy) then needs some 12-15 launches (35 ms) to return to
    its steady rate, while a plain read recovers in one; the timed region
    measures the steady rate."""
    import torch
    n = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(8):
            fn()
        n += 8
        stream.synchronize()
    return n


KERNEL_SOURCES = ("paper_1111_6661_amd/csrc/cube_device.h",
                  "paper_1111_6661_amd/csrc/cube_kernels.hip")
PROFILE_SUMMARY = "profiles/fused_brick16g_trace_and_bytes.md"
# Launch shapes the autotuner chose on an MI355X for the brick's pass kinds.
TUNE_TABLE = "paper_1111_6661_amd/tuning/gfx950.json"
# PCIe 5.0 x16, one direction: 32 GT/s x 16 lanes, 128b/130b coding.
PCIE_PEAK_GBS = 32e9 * 16 / 8 * 128 / 130 / 1e9


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per fused launch (FETCH + WRITE, scaled by the copy
    calibration) from the committed rocprofv3 summary -- only if it was taken
    on the current kernel sources, else None."""
    path = os.path.join(ROOT, PROFILE_SUMMARY)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    want = kernel_source_hash()
    if f"kernel sources sha256[:16]: {want}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return float(line.split(":", 1)[1])
    return None


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cube, nbins: int, lo: float, hi: float, target_s: float):
    """The oracle on the first planes of the cube, sized to about target_s,
    on one host core (the calling thread pinned to it while it runs)."""
    import oracle
    nz, ny, nx = cube.shape
    plane = nx * ny
    probe = cube[:1].cpu().numpy()
    old = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(old) if old else None
    try:
        if core is not None:
            os.sched_setaffinity(0, {core})
        t0 = time.perf_counter()
        oracle.stats(probe)
        oracle.hist(probe, lo, hi, nbins)
        per_plane = max(time.perf_counter() - t0, 1e-6)
        k = int(max(1, min(nz, target_s / per_plane)))
        sample = cube[:k].cpu().numpy()
        t0 = time.perf_counter()
        oracle.stats(sample)
        oracle.hist(sample, lo, hi, nbins)
        dt = time.perf_counter() - t0
    finally:
        if core is not None:
            os.sched_setaffinity(0, old)
    return {"value": k * plane / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} of {nz} channel planes ({k * plane} voxels): oracle stats "
                      f"(two sweeps) + histogram (one sweep), {dt:.1f} s single-threaded",
            "seconds": dt, "pinned_core": core, "cpu_model": _cpu_model(),
            "host_cores": os.cpu_count()}


def bench_batch64(cs, synth, torch, dev, steps: int, tune: bool = False):
    """64 uneven items, each statistics then a 512-bin histogram over its own
    [min, max]: one persistent launch replayed from a HIP graph, against the
    plain per-item calls (two launches each) on one stream.  The timed batch
    runs the automatic rule (the tuning table's, or a fresh autotune with
    `tune`); fixed tile sizes are swept beside it for context."""
    import numpy as np
    recs = synth.batch_item_recipes()
    items = [synth.cube_tensor(r, synth.BASE_SEED + 2 + i, device=dev) for i, r in enumerate(recs)]
    nvox = sum(r.n for r in recs)
    nb = synth.HIST_BINS["batch64"]
    n = len(items)
    stream = torch.cuda.Stream(device=dev)
    sp = stream.cuda_stream
    out = torch.zeros((n, 64), dtype=torch.uint8, device=dev)
    cnt = torch.zeros((n, nb + 3), dtype=torch.int64, device=dev)
    boxes = [cs.box_of(t) for t in items]
    qs = [cs.make_query(p, d, cs.CUBE_Q_MINMAX, nb, 0.0, 0.0, out[i].data_ptr(), cnt[i].data_ptr())
          for i, (p, d) in enumerate(boxes)]
    tuned = cs.cube_autotune_batch(qs, reps=5) if tune else None
    # fixed tile sizes beside the automatic rule (graph-replayed), for context
    tiles = {}
    for tv in (1 << 16, 1 << 17, 1 << 18, 1 << 20):
        b = cs.Batch(tile_voxels=tv)
        b.enqueue(qs, sp)
        b.check()
        _, ms = time_launches(lambda: b.graph_launch(sp), stream, max(5, steps // 3), 2)
        tiles[tv] = ms
        b.close()
    # the timed batch: automatic tile and threads (the tuned rule, if any)
    b = cs.Batch(tile_voxels=0, threads=0)
    b.enqueue(qs, sp)
    b.check()
    _, ev_b = time_launches(lambda: b.graph_launch(sp), stream, steps, 3)
    b.check()
    out2 = torch.zeros_like(out)
    cnt2 = torch.zeros_like(cnt)

    def plain():
        for i, (p, d) in enumerate(boxes):
            cs.cube_stats_hist_minmax_async(p, d, nb, out2[i].data_ptr(), cnt2[i].data_ptr(), sp)

    _, ev_p = time_launches(plain, stream, steps, 3)
    torch.cuda.synchronize()
    counts_equal = bool(torch.equal(cnt, cnt2))
    worst = 0.0
    for i in range(n):
        a = cs.Stats.from_bytes(out[i].cpu().numpy().tobytes())
        c = cs.Stats.from_bytes(out2[i].cpu().numpy().tobytes())
        if a.min != c.min or a.max != c.max or a.n_valid != c.n_valid:
            counts_equal = False
        worst = max(worst, abs(a.std - c.std) / c.std)
    b.close()
    del items
    return {"items": n, "voxels": nvox, "nbins": nb, "rule": "automatic (tuned rule if loaded)",
            "autotune": tuned,
            "fixed_tile_sweep_ms": {str(k): round(v, 4) for k, v in tiles.items()},
            "batched_graph_ms": ev_b, "plain_ms": ev_p,
            "batched_voxels_per_s": nvox / (ev_b * 1e-3), "plain_voxels_per_s": nvox / (ev_p * 1e-3),
            "speedup": ev_p / ev_b, "counts_and_extrema_equal": counts_equal,
            # two reads of every voxel (statistics, then the [min, max] histogram)
            "batched_gbs": 8 * nvox / (ev_b * 1e-3) / 1e9,
            "batched_frac_hbm_peak": 8 * nvox / (ev_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "max_std_rel_diff_batched_vs_plain": worst}


STRESS_ORACLE = "tests/golden/stress128g_oracle.json"


def stress_oracle_reference(synth):
    """The oracle's statistics of the whole stress cube, as stored by
    tests/golden/make_stress128g_oracle.py (read as data; the oracle is not
    run here), or None when the file is missing or was written for another
    generator or seed."""
    import hashlib
    path = os.path.join(ROOT, STRESS_ORACLE)
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    h = hashlib.sha256()
    for f in ("synth/__init__.py", "synth/gen.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if g.get("generator_sha256_16") != h.hexdigest()[:16] or g.get("seed") != synth.BASE_SEED + 4:
        return None
    return g["stats"]


def bench_stress(cs, synth, torch, dev, steps: int, tune: bool = False):
    """The precision-stress cube at full size (4096 x 4096 x 2048, 128 GiB,
    offset 1e4): fused pass throughput over [min, max] with 4096 bins, and
    the moments of the three accumulation modes side by side, with their
    errors relative to the oracle's values for the whole cube (stored with
    the tests; the test suite recomputes them live)."""
    name = "stress128g"
    r = synth.WORKLOADS[name]
    nb = synth.HIST_BINS[name]
    log(f"stress: generating {r.nx}x{r.ny}x{r.nz} ({r.n * 4 / 2**30:.0f} GiB)")
    cube = synth.cube_tensor(r, synth.BASE_SEED + 4, device=dev)
    ptr, dims = cs.box_of(cube)
    modes = {}
    for mode, label in ((cs.CUBE_ACCUM_NAIVE32, "naive32"), (cs.CUBE_ACCUM_KAHAN32, "kahan32"),
                        (cs.CUBE_ACCUM_FP64MERGE, "fp64merge")):
        cs.cube_set_accum_mode(mode)
        st = cs.stats(cube)
        modes[label] = {"mean": st.mean, "std": st.std}
    cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    st = cs.stats(cube)
    stream = torch.cuda.Stream(device=dev)
    sp = stream.cuda_stream
    out = torch.zeros(64, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(nb + 3, dtype=torch.int64, device=dev)
    lo, hi = st.min, st.max
    tuned = None
    if tune:
        tuned = cs.cube_autotune(cube.data_ptr(), dims, cs.CUBE_Q_FUSED, lo, hi, nb, reps=2)
        log(f"autotune (stress fused): {tuned['best']}")
    def fused():
        cs.cube_stats_hist_async(ptr, dims, lo, hi, nb, out.data_ptr(), cnt.data_ptr(), sp)

    prewarm(fused, stream, 150.0)
    _, ms = time_launches(fused, stream, steps, 2)
    c = cnt.cpu().numpy()
    plan = cs.cube_describe_plan(ptr, dims, cs.CUBE_Q_FUSED, nb)
    ref = modes["fp64merge"]
    orc = stress_oracle_reference(synth)
    vs_oracle = None
    if orc is not None and orc["n_valid"] == st.n_valid and orc["min"] == st.min \
            and orc["max"] == st.max:
        vs_oracle = {k: {"mean": abs(v["mean"] - orc["mean"]) / abs(orc["mean"]),
                         "std": abs(v["std"] - orc["std"]) / orc["std"]}
                     for k, v in modes.items()}
    del cube
    torch.cuda.empty_cache()
    return {"voxels": r.n, "nbins": nb, "fused_ms": ms, "voxels_per_s": r.n / (ms * 1e-3),
            "rel_err_vs_oracle": vs_oracle,
            "oracle_reference": STRESS_ORACLE if vs_oracle is not None else None,
            "autotune": tuned, "fused_plan": plan,
            "pct_hbm_peak": 100.0 * 4 * r.n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "bin0_fraction_of_valid": float(c[0]) / max(1, st.n_valid),
            "counts_sum_equals_n_total": int(c.sum()) == r.n,
            "mean_std_by_mode": modes,
            "std_rel_diff_vs_fp64merge": {k: abs(v["std"] - ref["std"]) / ref["std"]
                                          for k, v in modes.items()}}


def bench_serve(cs, synth, torch, dev, seconds: float, load_frac: float = 0.7,
                sweep=()):
    """Twelve resident cubes (about 201 GiB); a seeded Poisson query stream at
    load_frac of the plain server's closed-loop capacity, replayed against the
    plain server and the continuous-batching server (and the latter with a
    fixed 2^20-voxel tile).  Each load in `sweep` replays a stream of its own
    against plain and served."""
    import threading
    from paper_1111_6661_amd import workloads
    recipes = synth.serve_recipes()
    log(f"serve: generating {len(recipes)} cubes, "
        f"{sum(r.n for r in recipes) * 4 / 2**30:.1f} GiB")
    cubes = [synth.cube_tensor(r, synth.BASE_SEED + 3 + i, device=dev) for i, r in enumerate(recipes)]
    ranges = []
    for c in cubes:
        st = cs.stats(c)
        ranges.append(((st.min, st.max), (st.mean - 2 * st.std, st.mean + 2 * st.std)))
    shapes = [tuple(c.shape) for c in cubes]

    def make(specs):
        n = len(specs)
        out = torch.zeros((n, 64), dtype=torch.uint8, device=dev)
        cnt = torch.zeros((n, 4096 + 3), dtype=torch.int64, device=dev)
        qs = []
        for i, q in enumerate(specs):
            z0, z1, y0, y1, x0, x1 = q.box
            p, d = cs.box_of(cubes[q.cube][z0:z1, y0:y1, x0:x1])
            qs.append(cs.make_query(p, d, q.kind, q.nbins or 1, q.lo, q.hi, out[i].data_ptr(),
                                    cnt[i].data_ptr()))
        return qs, out, cnt

    def replay(mode, specs, open_loop: bool, tile: int = 0):
        qs, out, cnt = make(specs)
        srv = cs.Server(mode, slots=4, max_batch=32, max_inflight_bytes=1 << 30,
                        tile_voxels=tile)
        ids = [0] * len(qs)
        t0 = time.perf_counter()

        def submit_all():
            for i, q in enumerate(qs):
                if open_loop:
                    dt = specs[i].t_arrival - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                ids[i] = srv.submit(q)

        th = threading.Thread(target=submit_all)
        th.start()
        th.join()
        for i in ids:
            srv.wait(i)
        wall = time.perf_counter() - t0
        p50, p99, n = srv.latency()
        srv.close()
        torch.cuda.synchronize()
        return {"queries": n, "wall_s": wall, "p50_ms": p50 * 1e3, "p99_ms": p99 * 1e3,
                "qps": n / wall, "voxels_per_s": sum(q.voxels for q in specs) / wall}, out, cnt

    # closed-loop capacity of the plain server
    cap_specs = workloads.query_stream(shapes, ranges, 200, 1e9, synth.BASE_SEED + 30,
                                       cs.CUBE_Q_STATS, cs.CUBE_Q_FUSED)
    cap, _, _ = replay(cs.CUBE_SERVE_PLAIN, cap_specs, open_loop=False)
    qps = load_frac * cap["qps"]
    # at least 10^4 queries, so that p99 rests on about 100 samples above it
    n = max(MIN_SERVE_QUERIES, int(qps * seconds))
    specs = workloads.query_stream(shapes, ranges, n, qps, synth.BASE_SEED + 31,
                                   cs.CUBE_Q_STATS, cs.CUBE_Q_FUSED)
    log(f"serve: plain capacity {cap['qps']:.0f} QPS; replaying {n} queries at {qps:.0f} QPS")
    plain, po, pc = replay(cs.CUBE_SERVE_PLAIN, specs, open_loop=True)
    served, so, sc = replay(cs.CUBE_SERVE_BATCHED, specs, open_loop=True)
    # the first quarter of the same stream served with one fixed 2^20-voxel
    # tile for every query
    nf = max(50, n // 4)
    fixed, fo, fc = replay(cs.CUBE_SERVE_BATCHED, specs[:nf], open_loop=True, tile=1 << 20)
    same_counts = bool(torch.equal(pc, sc)) and bool(torch.equal(pc[:nf], fc))
    same_extrema = True
    po, so, fo = po.cpu(), so.cpu(), fo.cpu()
    for i in range(n):
        a = cs.Stats.from_bytes(po[i].numpy().tobytes())
        for o in ((so, fo) if i < nf else (so,)):
            b = cs.Stats.from_bytes(o[i].numpy().tobytes())
            if a.n_valid != b.n_valid or a.n_nan != b.n_nan or \
                    not (a.min == b.min or a.min != a.min) or not (a.max == b.max or a.max != a.max):
                same_extrema = False
    loads = {}
    for k, lf in enumerate(sweep):
        q2 = lf * cap["qps"]
        n2 = max(50, int(q2 * seconds))
        sp2 = workloads.query_stream(shapes, ranges, n2, q2, synth.BASE_SEED + 32 + k,
                                     cs.CUBE_Q_STATS, cs.CUBE_Q_FUSED)
        p2, _, pc2 = replay(cs.CUBE_SERVE_PLAIN, sp2, open_loop=True)
        s2, _, sc2 = replay(cs.CUBE_SERVE_BATCHED, sp2, open_loop=True)
        same_counts = same_counts and bool(torch.equal(pc2, sc2))
        loads[str(lf)] = {"offered_qps": q2, "queries": n2, "plain": p2, "served": s2}
        log(f"serve at {lf}x: plain p50/p99 {p2['p50_ms']:.2f}/{p2['p99_ms']:.2f} ms, "
            f"served {s2['p50_ms']:.2f}/{s2['p99_ms']:.2f} ms")
    del cubes
    torch.cuda.empty_cache()
    return {"cubes": len(recipes), "resident_gib": sum(r.n for r in recipes) * 4 / 2**30,
            "plain_capacity_qps": cap["qps"], "offered_qps": qps, "load_frac": load_frac,
            "queries": n, "plain": plain, "served": served,
            "served_fixed_tile_2e20": dict(fixed, note=f"first {nf} queries of the stream"),
            "p50_speedup": plain["p50_ms"] / served["p50_ms"],
            "p99_speedup": plain["p99_ms"] / served["p99_ms"],
            "load_sweep": loads,
            "results_equal_plain_vs_served": same_counts and same_extrema}


def bench_select(cs, torch, cube, n_valid: int, reps: int):
    """Exact selection of the lower middle and the median of the brick.

    Each selection reads the cube twice (two 4 B/voxel passes; the third pass
    reads only the candidates the second copied out, when they fit, as they
    do here); the calls are synchronous, so the times include their small host
    copies.  The
    selected value is checked by its rank: fewer than k+1 valid voxels lie
    below it and more than k lie at or below it.
    """
    k = (n_valid - 1) // 2
    v = cs.select(cube, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        v = cs.select(cube, k)
    sel_ms = (time.perf_counter() - t0) * 1e3 / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        m, nv = cs.median(cube)
    med_ms = (time.perf_counter() - t0) * 1e3 / reps
    # quantiles: the quartiles, and 64 levels at once (three or four reads
    # each, as the call's plan took them)
    qtimes, qreads = {}, {}
    for label, lv in (("quartiles", [0.25, 0.5, 0.75]),
                      ("levels64", [i / 63 for i in range(64)])):
        cs.quantiles(cube, lv)
        qreads[label] = cs.cube_last_quantile_reads()
        t0 = time.perf_counter()
        for _ in range(reps):
            qv, _ = cs.quantiles(cube, lv)
        qtimes[label] = round((time.perf_counter() - t0) * 1e3 / reps, 4)
    flat = cube.view(-1)
    below = int((flat < v).sum())
    at_or_below = int((flat <= v).sum())
    n = flat.numel()
    return {"rank": k, "value": v, "median": m, "n_valid": nv,
            "select_ms": round(sel_ms, 4), "median_ms": round(med_ms, 4),
            "select_gbs_2_passes": 2 * 4 * n / (sel_ms * 1e-3) / 1e9,
            "quantiles_ms": qtimes,
            "quantiles_reads": qreads,
            "quantiles_gbs": {kq: qreads[kq] * 4 * n / (v_ * 1e-3) / 1e9
                              for kq, v_ in qtimes.items()},
            "rank_property_holds": below <= k < at_or_below and nv == n_valid}


def bench_project(cs, torch, cube, stream, steps: int):
    """Channel-axis projections of the brick: maximum, FP64 sum and valid
    count per pixel in one read (4 B per voxel in, 16 B per pixel out)."""
    nz, ny, nx = cube.shape
    ptr, d = cs.box_of(cube)
    mip = torch.empty((ny, nx), dtype=torch.float32, device=cube.device)
    mom0 = torch.empty((ny, nx), dtype=torch.float64, device=cube.device)
    nv = torch.empty((ny, nx), dtype=torch.int32, device=cube.device)
    sp = stream.cuda_stream

    def run():
        cs.cube_project(ptr, d, mip.data_ptr(), mom0.data_ptr(), nv.data_ptr(), sp)

    _, ev = time_launches(run, stream, steps, 2)
    torch.cuda.synchronize()
    nbytes = 4 * cube.numel() + 16 * nx * ny
    gbs = nbytes / (ev * 1e-3) / 1e9
    return {"ms": round(ev, 4), "gbs": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
            "bytes_per_call": nbytes, "valid_total": int(nv.to(torch.int64).sum())}


def bench_host(cs, torch, cube, lo: float, hi: float, nbins: int, planes: int, reps: int):
    """Out-of-core fused queries over a copy of the brick's first planes in
    host memory: pinned (hipHostMalloc through torch) and pageable (numpy).
    The link ceiling is a plain 1 GiB pinned host-to-device copy."""
    import numpy as np
    sub = cube[:planes]
    n = sub.numel()
    pinned = torch.empty(tuple(sub.shape), dtype=torch.float32, pin_memory=True)
    pinned.copy_(sub)
    dst = torch.empty(1 << 28, dtype=torch.float32, device=cube.device)
    src = pinned.view(-1)[:1 << 28]
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    copy_gbs = 3 * 4 * (1 << 28) / (time.perf_counter() - t0) / 1e9
    del dst
    st_d, cnt_d = cs.stats_hist(sub, lo, hi, nbins)
    res = {"planes": planes, "voxels": n, "bytes": 4 * n, "link_copy_gbs": copy_gbs,
           "link_peak_gbs": PCIE_PEAK_GBS}
    for label, arr in (("pinned", pinned), ("pageable", None)):
        if arr is None:
            arr = pinned.numpy().copy()
        cs.host_query(arr, cs.CUBE_Q_FUSED, nbins, lo, hi)   # warm-up
        t0 = time.perf_counter()
        for _ in range(reps):
            st, cnt = cs.host_query(arr, cs.CUBE_Q_FUSED, nbins, lo, hi)
        dt = (time.perf_counter() - t0) / reps
        res[label] = {"s_per_query": dt, "gbs": 4 * n / dt / 1e9,
                      "frac_of_copy": 4 * n / dt / 1e9 / copy_gbs,
                      "counts_equal_resident": bool(np.array_equal(cnt, cnt_d)),
                      "extrema_equal_resident": st.min == st_d.min and st.max == st_d.max,
                      "std_rel_diff_vs_resident": abs(st.std - st_d.std) / st_d.std}
        del arr
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--launch", default="",
                    help="threads,blocks,hist_copies,unroll override (0 = automatic)")
    ap.add_argument("--only-fused", action="store_true",
                    help="time the fused pass only (for profiler runs)")
    ap.add_argument("--tune", choices=("table", "run", "batch", "off"), default="table",
                    help="launch shapes: the shipped tuning table (autotune if it is "
                         "missing), a fresh autotune of every class, the table with a fresh "
                         "autotune of the batched launch's rule only, or the planner's defaults")
    ap.add_argument("--tune-save", default="", help="save the tuning table to this path")
    ap.add_argument("--tune-table", default="",
                    help="tuning table to load instead of the shipped one")
    ap.add_argument("--no-tune", action="store_true", help="same as --tune off")
    ap.add_argument("--prewarm-ms", type=float, default=150.0,
                    help="untimed fused launches for this long before the warm-up steps "
                         "(the shader clock's ramp after idle; 0 = none)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-item batch")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-stress", action="store_true", help="skip the 128 GiB stress cube")
    ap.add_argument("--no-select", action="store_true", help="skip selection and median")
    ap.add_argument("--no-host", action="store_true", help="skip the out-of-core host queries")
    ap.add_argument("--only-stress", action="store_true",
                    help="time the 128 GiB stress cube's fused pass only and print its record "
                         "(for profiler runs; not the benchmark line)")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the replayed query stream (at least 10^4 queries)")
    ap.add_argument("--serve-sweep", default="",
                    help="more offered loads (fractions of the plain capacity), e.g. 0.5,0.9")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (a cube would "
              "shard by channel slabs with one all-gather of per-GPU records); "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1111_6661_amd as cs
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.launch:
        cs.cube_set_launch(*[int(v) for v in args.launch.split(",")])
    if args.only_stress:
        table = os.path.join(ROOT, TUNE_TABLE)
        if not (args.no_tune or args.launch) and os.path.exists(table):
            cs.cube_tune_load(table)
        rec = bench_stress(cs, synth, torch, dev, args.steps)
        print(json.dumps({"stress128g": rec}), flush=True)
        return 0
    name = "brick16g"
    r = synth.WORKLOADS[name]
    nbins = synth.HIST_BINS[name]
    log(f"generating {name} {r.nx}x{r.ny}x{r.nz} ({r.n * 4 / 2**30:.1f} GiB)")
    t0 = time.perf_counter()
    cube = synth.cube_tensor(r, synth.BASE_SEED + 1, device=dev)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    ptr, dims = cs.box_of(cube)

    st0 = cs.stats(cube)
    lo, hi = float(st0.min), float(st0.max)
    log(f"stats: n_nan={st0.n_nan} min={lo} max={hi} mean={st0.mean:.6g} std={st0.std:.6g}")

    tuned = None
    mode = "off" if (args.no_tune or args.launch) else args.tune
    table = args.tune_table or os.path.join(ROOT, TUNE_TABLE)
    if mode in ("table", "batch") and os.path.exists(table):
        tuned = {"source": args.tune_table or TUNE_TABLE, "entries": cs.cube_tune_load(table)}
        log(f"tuning table {TUNE_TABLE}: {tuned['entries']} entries")
    elif mode != "off":
        tuned = {"source": "autotune"}
        for kname, kind in (("fused", cs.CUBE_Q_FUSED), ("stats", cs.CUBE_Q_STATS),
                            ("hist", cs.CUBE_Q_HIST)):
            tuned[kname] = cs.cube_autotune(cube.data_ptr(), dims, kind, lo, hi, nbins, reps=4)
            log(f"autotune ({kname}): {tuned[kname]['best']}")

    stream = torch.cuda.Stream(device=dev)
    out = torch.zeros(64, dtype=torch.uint8, device=dev)
    counts = torch.zeros(nbins + 3, dtype=torch.int64, device=dev)
    sp = stream.cuda_stream

    def fused():
        cs.cube_stats_hist_async(ptr, dims, lo, hi, nbins, out.data_ptr(), counts.data_ptr(), sp)

    def stats_only():
        cs.cube_stats_async(ptr, dims, out.data_ptr(), sp)

    def hist_only():
        cs.cube_hist_async(ptr, dims, lo, hi, nbins, counts.data_ptr(), sp)

    def two_pass():
        cs.cube_stats_hist_minmax_async(ptr, dims, nbins, out.data_ptr(), counts.data_ptr(), sp)

    probe_word = torch.zeros(1, dtype=torch.int32, device=dev)

    def read_probe():
        # the fused pass's reads alone (same launch shape and order)
        cs.cube_read_probe(ptr, dims, nbins, probe_word.data_ptr(), sp)

    # A plain copy of known size (1 GiB read + 1 GiB written), outside the
    # timed region: profiler byte counters are scaled by what they read for it.
    cal_src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst

    stream.wait_stream(torch.cuda.current_stream())
    n_prewarm = prewarm(fused, stream, args.prewarm_ms) if args.prewarm_ms > 0 else 0
    log(f"prewarm: {n_prewarm} untimed fused launches ({args.prewarm_ms:.0f} ms)")
    # The timed region: exactly `steps` fused launches, bracketed by syncs.
    torch.cuda.synchronize()
    wall_ms, ev_ms = time_launches(fused, stream, args.steps, args.warmup)
    torch.cuda.synchronize()
    ev_median_ms = float(np.median(time_launches.last))
    st = cs.Stats.from_bytes(out.cpu().numpy().tobytes())
    c = counts.cpu().numpy().view(np.uint64)
    log(f"fused: {ev_ms:.4f} ms/launch (events), {wall_ms:.4f} ms/step wall")
    parity = {
        "counts_sum_equals_n_total": int(c.sum()) == st.n_total,
        "below_above_zero_over_minmax": int(c[nbins]) == 0 and int(c[nbins + 1]) == 0,
        "extrema_equal_stats_pass": st.min == st0.min and st.max == st0.max,
        "nan_equals_stats_pass": int(c[nbins + 2]) == st0.n_nan == st.n_nan,
    }

    extra = {"fused_plan": cs.cube_describe_plan(ptr, dims, cs.CUBE_Q_FUSED, nbins),
             "prewarm": {"ms": args.prewarm_ms, "launches": n_prewarm,
                         "why": "untimed launches before the warm-up steps: the shader clock "
                                "ramps back up over about 35 ms of the fused pass after idle"}}
    log(f"fused plan: {extra['fused_plan']}")
    n_short = max(5, args.steps // 2)
    _, probe_ms = time_launches(read_probe, stream, n_short, 2)
    probe_gbs = 4 * r.n / (probe_ms * 1e-3) / 1e9
    extra["read_probe"] = {"ms_per_call_events": round(probe_ms, 4), "gbs": probe_gbs,
                           "frac_hbm_peak": probe_gbs / HBM_PEAK_GBS,
                           "fused_frac_of_probe": probe_ms / ev_ms}
    log(f"read probe: {probe_ms:.4f} ms ({probe_gbs:.0f} GB/s); fused reaches "
        f"{100 * probe_ms / ev_ms:.1f} % of it")
    others = () if args.only_fused else (("stats_only", stats_only), ("hist_only", hist_only),
                                          ("two_pass_minmax", two_pass))
    for label, fn in others:
        w, e = time_launches(fn, stream, n_short, 2)
        extra[label] = {"ms_per_call_events": round(e, 4), "voxels_per_s": r.n / (e * 1e-3)}
        log(f"{label}: {e:.4f} ms")

    if tuned is not None:
        extra["tuning"] = tuned
    if not args.only_fused and not args.no_batch:
        log("batch64 ...")
        extra["batch64"] = bench_batch64(cs, synth, torch, dev, max(10, args.steps // 2),
                                         tune=mode in ("run", "batch"))
        log(f"batch64: graph {extra['batch64']['batched_graph_ms']:.3f} ms vs plain "
            f"{extra['batch64']['plain_ms']:.3f} ms")
    if not args.only_fused and not args.no_select:
        sel = bench_select(cs, torch, cube, int(st0.n_valid), 5)
        extra["select_median"] = sel
        parity["median_rank_property"] = sel["rank_property_holds"]
        log(f"select: {sel['select_ms']:.3f} ms, median: {sel['median_ms']:.3f} ms, "
            f"quantiles: {sel['quantiles_ms']}")
    if not args.only_fused:
        pj = bench_project(cs, torch, cube, stream, n_short)
        extra["project"] = pj
        parity["project_valid_total_equals_stats"] = pj.pop("valid_total") == st0.n_valid
        log(f"project: {pj['ms']:.3f} ms ({100 * pj['frac_hbm_peak']:.1f} % of HBM peak)")
    if not args.only_fused and not args.no_host:
        hq = bench_host(cs, torch, cube, lo, hi, nbins, 256, 3)
        extra["host_out_of_core"] = hq
        parity["host_counts_equal_resident"] = (hq["pinned"]["counts_equal_resident"] and
                                                hq["pageable"]["counts_equal_resident"])
        log(f"host streaming: pinned {hq['pinned']['gbs']:.1f} GB/s, pageable "
            f"{hq['pageable']['gbs']:.1f} GB/s, plain copy {hq['link_copy_gbs']:.1f} GB/s")
    bytes_per_launch = 4 * r.n
    achieved = bytes_per_launch / (ev_ms * 1e-3) / 1e9
    value = r.n / (wall_ms * 1e-3)
    result = {
        "metric": "fused stats+histogram voxels/s (% of HBM peak); p50/p99 query latency",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: float32 cube {r.nx}x{r.ny}x{r.nz} (16 GiB), noise + "
                               f"{r.n_sources} sources, 1% NaN, fused stats + {nbins}-bin "
                               f"histogram over [min, max]",
                   "nbins": nbins, "voxels": r.n},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(),
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "read_probe_gbs": probe_gbs,
                     "frac_of_read_probe": achieved / probe_gbs,
                     "kernel_sources": kernel_source_hash()},
        "pct_hbm_peak": 100.0 * achieved / HBM_PEAK_GBS,
        "kernel_ms_events": ev_ms,
        "kernel_ms_events_median": ev_median_ms,
        "parity": parity,
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(cube, nbins, lo, hi, args.cpu_seconds)
        result["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['value']:.3g} voxels/s")
    if not args.only_fused and not args.no_stress:
        del cube
        cube = None
        torch.cuda.empty_cache()
        extra["stress128g"] = bench_stress(cs, synth, torch, dev, 10, tune=mode == "run")
        log(f"stress128g: fused {extra['stress128g']['fused_ms']:.3f} ms "
            f"({extra['stress128g']['pct_hbm_peak']:.1f} % of HBM peak)")
    if not args.only_fused and not args.no_serve:
        cube = None
        torch.cuda.empty_cache()
        sweep = [float(v) for v in args.serve_sweep.split(",") if v.strip()]
        sv = bench_serve(cs, synth, torch, dev, args.serve_seconds, sweep=sweep)
        extra["serve"] = sv
        result["p50_ms"] = sv["served"]["p50_ms"]
        result["p99_ms"] = sv["served"]["p99_ms"]
        log(f"serve: plain p50/p99 {sv['plain']['p50_ms']:.2f}/{sv['plain']['p99_ms']:.2f} ms, "
            f"served {sv['served']['p50_ms']:.2f}/{sv['served']['p99_ms']:.2f} ms, "
            f"fixed 2^20 tile {sv['served_fixed_tile_2e20']['p50_ms']:.2f}/"
            f"{sv['served_fixed_tile_2e20']['p99_ms']:.2f} ms")
    if args.tune_save:
        cs.cube_tune_save(args.tune_save)
    # release everything before the line is printed: no device or pinned
    # memory, stream or library thread outlives the measurement
    cube = None
    torch.cuda.synchronize()
    cs.cube_shutdown()
    torch.cuda.empty_cache()
    print(json.dumps(result), flush=True)
    return 0 if all(parity.values()) else 1


if __name__ == "__main__":
    sys.exit(main())
