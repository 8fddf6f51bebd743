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
              on the launch stream, against the 8 TB/s HBM peak;
  cpu_baseline the oracle (single thread) on a bounded sample of the cube;
  extra       two-pass [min, max] timings, stats-only and histogram-only
              kernel timings, and the parity of the timed result.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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
    ev = sum(a.elapsed_time(b) for a, b in evs) / steps
    return wall, ev


def cpu_baseline(cube, nbins: int, lo: float, hi: float, target_s: float):
    """The oracle on the first planes of the cube, sized to about target_s."""
    import oracle
    nz, ny, nx = cube.shape
    plane = nx * ny
    probe = cube[:1].cpu().numpy()
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
    return {"value": k * plane / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} of {nz} channel planes ({k * plane} voxels): oracle stats "
                      f"(two sweeps) + histogram (one sweep), {dt:.1f} s single-threaded",
            "seconds": dt}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1111_6661_amd as cs
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.launch:
        cs.cube_set_launch(*[int(v) for v in args.launch.split(",")])
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

    stream.wait_stream(torch.cuda.current_stream())
    # The timed region: exactly `steps` fused launches, bracketed by syncs.
    torch.cuda.synchronize()
    wall_ms, ev_ms = time_launches(fused, stream, args.steps, args.warmup)
    torch.cuda.synchronize()
    st = cs.Stats.from_bytes(out.cpu().numpy().tobytes())
    c = counts.cpu().numpy().view(np.uint64)
    log(f"fused: {ev_ms:.4f} ms/launch (events), {wall_ms:.4f} ms/step wall")
    parity = {
        "counts_sum_equals_n_total": int(c.sum()) == st.n_total,
        "below_above_zero_over_minmax": int(c[nbins]) == 0 and int(c[nbins + 1]) == 0,
        "extrema_equal_stats_pass": st.min == st0.min and st.max == st0.max,
        "nan_equals_stats_pass": int(c[nbins + 2]) == st0.n_nan == st.n_nan,
    }

    extra = {}
    n_short = max(5, args.steps // 2)
    others = () if args.only_fused else (("stats_only", stats_only), ("hist_only", hist_only),
                                          ("two_pass_minmax", two_pass))
    for label, fn in others:
        w, e = time_launches(fn, stream, n_short, 2)
        extra[label] = {"ms_per_call_events": round(e, 4), "voxels_per_s": r.n / (e * 1e-3)}
        log(f"{label}: {e:.4f} ms")

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
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "pct_hbm_peak": 100.0 * achieved / HBM_PEAK_GBS,
        "kernel_ms_events": ev_ms,
        "parity": parity,
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(cube, nbins, lo, hi, args.cpu_seconds)
        result["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['value']:.3g} voxels/s")
    print(json.dumps(result), flush=True)
    return 0 if all(parity.values()) else 1


if __name__ == "__main__":
    sys.exit(main())
