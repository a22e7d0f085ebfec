"""Build libgosma.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1812_01232_amd.build [-v]
"""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libgosma.so"
SOURCES = ["api.hip", "bound.hip", "bb.hip", "mlp.hip", "tune.hip", "sma.hip", "mixgen.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# gfx950 only; packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


# Per-file flags: the clustering decisions of mixgen.hip must be the plain
# left-to-right FP64 expressions (no fused multiply-adds).
FILE_FLAGS = {"mixgen.hip": ["-ffp-contract=off"]}


def build(verbose=False, extra=()):
    build_dir = PKG / "_build"
    build_dir.mkdir(exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = build_dir / (src + ".o")
        cmd = [HIPCC, *DEVICE_FLAGS, *FILE_FLAGS.get(src, []), *extra, "-I", str(ROOT / "include"), "-I", str(CSRC),
               "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(str(obj))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
