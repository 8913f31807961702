"""Build libfr.so (HIP kernels + C ABI) for gfx950, in-tree, with hipcc.

Each source is compiled to an object in parallel (the kernel files take a minute or more each),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfr.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("fr_kernels.hip", "fr_kernels32.hip", "fr_mlp.hip", "fr_partition.hip",
                                                  "fr_host.cpp")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-I" + os.path.join(ROOT, "include"),
    # packed FP32 instructions stay off on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-pthread",
]


def object_path(src: str) -> str:
    return os.path.join(OBJ_DIR, os.path.basename(src) + ".o")


def compile_command(src: str) -> list:
    return ["hipcc", *FLAGS, "-c", "-o", object_path(src), src]


def link_command(out: str = LIB) -> list:
    return ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", out,
            *[object_path(s) for s in SOURCES]]


def hipcc_command(out: str = LIB) -> list:
    """The equivalent single-command build (all sources at once)."""
    return ["hipcc", *FLAGS, "-shared", "-o", out, *SOURCES]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        for f in [ex.submit(run, compile_command(s)) for s in SOURCES]:
            f.result()
    tmp = LIB + ".tmp"
    run(link_command(tmp))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
