"""Builds librendermap.so (HIP for gfx950) in-tree with hipcc, and beside it
librm_microbench.so, the atomic-throughput microbenchmarks the benchmark
reports as secondary ceilings (not part of the library)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "librendermap.so"
SOURCES = ["rm_api.cpp", "rm_mesh.hip", "rm_raster.hip", "rm_optim.hip", "rm_icp.hip", "rm_noalloc.hip"]
MB_LIB = PKG / "librm_microbench.so"
MB_SOURCES = ["rm_microbench.hip"]

# -ffp-contract=off: every float operation is the single IEEE operation
# written (the rasterization contract uses explicit fmaf); packed FP32
# instructions are disabled for the whole library.
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


def _link(hipcc: str, out: Path, sources, verbose: bool) -> None:
    tmp = out.with_suffix(".so.tmp")
    cmd = [hipcc, *FLAGS, "-o", str(tmp), *[str(CSRC / s) for s in sources]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> Path:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    _link(hipcc, LIB, SOURCES, verbose)
    _link(hipcc, MB_LIB, MB_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB, file=sys.stderr)
