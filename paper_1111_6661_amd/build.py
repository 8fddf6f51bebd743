"""Compile the HIP library ``libcubestats.so`` for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcubestats.so")
SOURCES = ["cube_kernels.hip", "cube_capi.hip", "cube_batch.hip", "cube_server.hip", "cube_tune.hip",
           "cube_select.hip", "cube_host.hip",
           "cube_project.hip"]

# -packed-fp32-ops: no packed FP32 instructions are emitted (the kernels are
# written for scalar FP32 VALU operations only).  -ffp-contract=off: no
# multiply-add contraction other than the explicit fmaf calls; denormals are
# kept (no -fgpu-flush-denormals-to-zero).
HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fvisibility=hidden",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-result", "-Wno-unused-value"]


def build(verbose: bool = False) -> str:
    """Always recompiles; returns the path of the library."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed:\n{out}")
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
