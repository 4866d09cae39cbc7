"""Builds the gfx950 HIP library ``liblbm_hip.so`` in-tree with hipcc.

Usage: ``python -m paper_2506_21804_amd.build`` (or ``build()`` from Python).
Every source is compiled as HIP for gfx950 only, C++20, -O3, with the packed
FP32 instructions disabled (``-packed-fp32-ops``): the compiler keeps plain
scalar FP32 arithmetic.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["abi.cpp", "geometry.cpp", "revolve.cpp", "kernels.hip", "adjoint.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


BUILD_DIR = os.path.join(HERE, "_build")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
         "-I", os.path.join(HERE, "..", "include")]


def compile_command(src: str, obj: str) -> list:
    return [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs: list, out: str) -> list:
    return [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out]


def build(verbose: bool = False) -> str:
    """Compiles the library (always, even when a built copy exists); sources
    compile in parallel, then one link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = [os.path.join(BUILD_DIR, s + ".o") for s in SOURCES]
    cmds = [compile_command(s, o) for s, o in zip(SOURCES, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, r in zip(cmds, results):
        if r.stderr:
            sys.stderr.write("\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l) + "\n")
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, c)
    tmp = LIB + ".tmp"
    subprocess.run(link_command(objs, tmp), check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
