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


# host-side sanitizers only (the device code is not instrumented): each flag behind -Xarch_host
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def object_path(src: str, san: bool = False) -> str:
    return os.path.join(OBJ_DIR, ("san_" if san else "") + os.path.basename(src) + ".o")


def compile_command(src: str, san: bool = False) -> list:
    return ["hipcc", *FLAGS, *(SAN_FLAGS if san else []), "-c", "-o", object_path(src, san), src]


def link_command(out: str = LIB, san: bool = False) -> list:
    return ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *(SAN_FLAGS if san else []),
            "-o", out, *[object_path(s, san) for s in SOURCES]]


def hipcc_command(out: str = LIB) -> list:
    """The equivalent single-command build (all sources at once)."""
    return ["hipcc", *FLAGS, "-shared", "-o", out, *SOURCES]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Build libfr.so; sanitize=True builds _build/libfr_san.so instead, with the host code under
    the address and undefined-behaviour sanitizers (load it with FR_LIB_PATH, the clang ASan
    runtime preloaded)."""
    os.makedirs(OBJ_DIR, exist_ok=True)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        for f in [ex.submit(run, compile_command(s, sanitize)) for s in SOURCES]:
            f.result()
    out = os.path.join(OBJ_DIR, "libfr_san.so") if sanitize else LIB
    tmp = out + ".tmp"
    run(link_command(tmp, sanitize))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
