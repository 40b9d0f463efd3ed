"""Build the HIP library ``libls_ed.so`` (gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only; packed FP32 instructions are
disabled (``-packed-fp32-ops``); no fast-math, so FP64 division and square
root round correctly; no floating-point contraction (``-ffp-contract=off``):
a multiply-add is fused only where the source writes fma(), so two kernels
built from the same row code (the single and the persistent batched launch)
round identically whatever their register budgets and block layouts.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libls_ed.so")
SOURCES = ["api.cpp", "group.cpp", "terms.cpp", "basis.hip", "matvec.hip", "batch.hip", "lanczos.hip", "stored.hip"]
HEADERS = ["ls_internal.hpp", "orbit.hpp", "matvec_impl.hpp", "dispatch.hpp"]

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off",
          "-Wall", "-Wno-unused-function"]


def _scratch_kernels(remarks: str):
    """Kernels whose resource-usage remark reports scratch (register spills
    to memory) or a stack whose size is only known at run time (which the
    runtime would have to guess), from hipcc's
    -Rpass-analysis=kernel-resource-usage output."""
    out = []
    for block in re.split(r"remark: Function Name: ", remarks)[1:]:
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", block)
        if m and int(m.group(1)) > 0:
            out.append((block.split()[0], int(m.group(1))))
        if re.search(r"Dynamic Stack: True", block):
            out.append((block.split()[0], "dynamic stack"))
    return out


def _compile(src: str) -> str:
    out = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-c", os.path.join(CSRC, src), "-o", out] + COMMON
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # every kernel must run from registers: a spill costs a memory round trip
    # per access inside the element loop
    spills = _scratch_kernels(r.stderr)
    if spills:
        raise RuntimeError(f"{src}: kernels spill to scratch: {spills}")
    return out


def build(jobs: int = 6, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-o", tmp, f"--offload-arch={ARCH}"] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
