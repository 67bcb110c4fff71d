"""Build ``libmehdg.so`` in-tree with hipcc for gfx950.

    python -m paper_2507_22195_amd.build

The library is three translation units: ``csrc/mehdg_api.hip`` (hexahedral
macro-elements, every kernel family of the step), ``csrc/mehdg_tet.hip``
(tetrahedral macro-elements) and ``csrc/mehdg_batch.hip`` (mixed-degree
batches over per-degree contexts, host code).  Packed FP32 instructions are disabled for all device
code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmehdg.so")
ARCH = os.environ.get("MEHDG_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, "mehdg_api.hip"), os.path.join(CSRC, "mehdg_tet.hip"),
            os.path.join(CSRC, "mehdg_batch.hip")]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmehdg.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
