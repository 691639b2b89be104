"""Builds ``libtl.so`` (the C-ABI library of HIP kernels) for gfx950 in-tree.

    python -m paper_1804_10120_amd.build

The library is compiled with hipcc for gfx950 only.  Packed FP32 instructions
are disabled (all arithmetic here is FP64 anyway).  The compiler's per-kernel
resource report (VGPRs, SGPRs, scratch, occupancy) is written beside the
objects in ``_build/resource_usage.txt``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtl.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["tl_kernels.hip", "tl_expr.hip", "generated/tlg_kernels.hip", "tl_abi.cpp"]
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r


def build(verbose: bool = False) -> str:
    """Regenerates the generated kernels from the registry, compiles every
    translation unit (in parallel) and links libtl.so."""
    from .codegen.__main__ import main as codegen
    codegen([])
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        results = list(pool.map(lambda s: _compile(s, verbose), SOURCES))
    objs, report = [], []
    for src, obj, r in results:
        report.append(r.stderr)
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(os.path.join(BUILD, "resource_usage.txt"), "w") as f:
        f.write("".join(report))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
