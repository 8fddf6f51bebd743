"""Compile the HIP library ``libcubestats.so`` for gfx950 (in-tree).

Each source is compiled to an object in parallel (a temporary directory),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcubestats.so")
SOURCES = ["cube_kernels.hip", "cube_capi.hip", "cube_batch.hip", "cube_server.hip",
           "cube_tune.hip", "cube_select.hip", "cube_host.hip", "cube_project.hip", "cube_probe.hip",
           "cube_quantile.hip", "cube_noalloc.hip"]

# -packed-fp32-ops: no packed FP32 instructions are emitted (the kernels are
# written for scalar FP32 VALU operations only).  -ffp-contract=off: no
# multiply-add contraction other than the explicit fmaf calls; denormals are
# kept (no -fgpu-flush-denormals-to-zero).
HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
               "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fvisibility=hidden",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-result", "-Wno-unused-value"]


def _run(cmd) -> str:
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed: {' '.join(cmd[-3:])}\n{out}")
    return out


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Always recompiles; returns the path of the library."""
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="cubestats_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [["hipcc", *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            outs = list(ex.map(_run, cmds))
        tmp = LIB + ".tmp"
        outs.append(_run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]))
    if verbose:
        text = "\n".join(o for o in outs if o.strip())
        if text:
            print(text)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
