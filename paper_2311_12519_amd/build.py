"""Build libhyena.so (the gfx950 HIP library) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, then linked into ``paper_2311_12519_amd/libhyena.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhyena.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["params.cpp", "crypto.cpp", "plan.cpp", "ntt.hip", "conv.hip", "synth.hip", "direct.hip", "client.hip", "simd.hip", "batch.hip", "mlp.hip", "calib.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "--offload-arch=gfx950", "-O3", "-fPIC", "-Wall", "-Wextra", "-Werror",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


# The NTT keeps each thread's residues in registers, which needs its fully
# unrolled butterfly nests (up to 64 residues x 6 stages) to stay unrolled;
# LLVM's default size cap for `#pragma unroll` would leave the largest one
# rolled and the register array on the scratch stack.
EXTRA = {"ntt.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    vs = os.path.join(BUILD_DIR, "exports.map")
    with open(vs, "w") as f:
        f.write("{ global: hyena_*; local: *; };\n")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread",
           "-Wl,--version-script=" + vs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
