"""Build libfr.so (HIP kernels + C ABI) for gfx950, in-tree, with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfr.so")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("fr_kernels.hip", "fr_kernels32.hip", "fr_mlp.hip", "fr_host.cpp")]


def hipcc_command(out: str = LIB) -> list:
    return [
        "hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-I" + os.path.join(ROOT, "include"),
        # packed FP32 instructions stay off on this target
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-pthread", "-o", out, *SOURCES,
    ]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
