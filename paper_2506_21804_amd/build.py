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
SOURCES = ["abi.cpp", "geometry.cpp", "revolve.cpp", "spread.cpp", "kernels.hip", "adjoint.hip"]
# adjoint.hip is compiled once more per (lattice, storage) pair, each copy
# holding that pair's adjoint kernels (ADJ_PART), so that they build in parallel
ADJOINT_PARTS = 6
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


BUILD_DIR = os.path.join(HERE, "_build")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
         "-I", os.path.join(HERE, "..", "include")]


def compile_command(src: str, obj: str, extra=()) -> list:
    return [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]


def units() -> list:
    """(source, object, extra flags) of every compilation unit."""
    out = [(s, os.path.join(BUILD_DIR, s + ".o"), ()) for s in SOURCES]
    out += [("adjoint.hip", os.path.join(BUILD_DIR, f"adjoint.part{k}.o"), (f"-DADJ_PART={k}",))
            for k in range(ADJOINT_PARTS)]
    return out


def link_command(objs: list, out: str) -> list:
    return [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out]


def build(verbose: bool = False) -> str:
    """Compiles the library (always, even when a built copy exists); sources
    compile in parallel, then one link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    us = units()
    objs = [o for _, o, _ in us]
    cmds = [compile_command(s, o, e) for s, o, e in us]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 4)) as ex:
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
