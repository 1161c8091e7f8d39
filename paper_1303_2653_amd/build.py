"""Compile the HIP library for gfx950 in-tree: paper_1303_2653_amd/liblbdps.so."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", "lbdps.hip")]
DEPS = [os.path.join(HERE, "csrc", f) for f in ("device.hpp", "kernels.hpp", "batch.hpp", "lattice3d.hpp", "coupled3d.hpp", "spheres_tile.hpp")] + [os.path.join(ROOT, "include", "lbdps.h")]
LIB = os.path.join(HERE, "liblbdps.so")

# -ffp-contract=off: no fused multiply-add contraction, so FP64 results follow the
# written evaluation order.  Packed FP32 instructions are disabled for gfx950.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-Wno-pass-failed"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(force: bool = True) -> str:
    newest = max(os.path.getmtime(p) for p in SRC + DEPS)
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= newest:
        return LIB
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", LIB + ".tmp", *SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv or True))
