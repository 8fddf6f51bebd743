"""Write the oracle's statistics of the 128 GiB precision-stress cube.

The cube (4096 x 4096 x 2048 float32, 2^35 voxels, offset 1e4, noise 1e-3,
10^5 sources, 2 % blank) is generated on the GPU by the seeded input
generator, streamed to the host slab by slab and swept by the oracle on host
threads (tests/devstream.py); nothing else computes these values.  The JSON
names the recipe, the seed and a hash of the generator's sources, so a reader
can tell when the stored values no longer describe the cube the generator
makes.

Usage (needs a GPU with 128 GiB free):
    python tests/golden/make_stress128g_oracle.py [OUT.json]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stress128g_oracle.json")


def generator_hash() -> str:
    h = hashlib.sha256()
    for f in ("synth/__init__.py", "synth/gen.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main() -> int:
    import dataclasses

    import torch

    import oracle
    import synth
    from tests.devstream import SLAB_PLANES, host_threads, oracle_stats_of_device

    out = sys.argv[1] if len(sys.argv) > 1 else OUT
    r = synth.WORKLOADS["stress128g"]
    seed = synth.BASE_SEED + 4
    t = synth.cube_tensor(r, seed, device="cuda")
    threads = host_threads()
    print(f"oracle over {r.n} voxels on {threads} threads ...", flush=True)
    t0 = time.perf_counter()
    ref = oracle_stats_of_device(oracle, t, threads)
    dt = time.perf_counter() - t0
    rec = {"workload": "stress128g", "recipe": dataclasses.asdict(r), "seed": seed,
           "generator_sha256_16": generator_hash(), "slab_planes": SLAB_PLANES,
           "oracle_seconds": round(dt, 1), "threads": threads,
           "stats": dataclasses.asdict(ref)}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec["stats"]), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
