"""Build libqvec.so (the HIP library behind include/sv.h) for gfx950 with hipcc.

Run ``python -m paper_2508_15545_amd.build`` (or call ``build()``); the
library lands next to this file, in-tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqvec.so")
SOURCES = ["kernels.hip", "kernels_block_c128.hip", "kernels_block_c64.hip", "gates.cpp", "planner.cpp", "capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are kept off: the compiler must not form them.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def _compile_cmd(src: str, obj: str) -> list:
    path = os.path.join(CSRC, src)
    lang = ["-x", "hip"]  # every source goes through the HIP driver (kernels and host API)
    return [HIPCC, *COMMON, *DEVICE_FLAGS, *lang, "-c", path, "-o", obj]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one process per source) and link
    libqvec.so. Always recompiles."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = _compile_cmd(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *DEVICE_FLAGS, "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
