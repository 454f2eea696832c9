"""Compile the HIP library libdcrf.so for gfx950 (in-tree).

Every translation unit is compiled separately with hipcc (in parallel), then
linked into ``paper_1608_06192_amd/libdcrf.so``. Flags:

* ``--offload-arch=gfx950 -O3``
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 math is
  generated from ordinary float code;
* ``-ffp-contract=off`` for lattice.hip only: the lattice coordinates are
  evaluated without fused multiply-adds, so the vertex set is the one a plain
  IEEE evaluation of the same formulas gives.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdcrf.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result", "-Wno-pass-failed",
]

SOURCES = {
    "lattice.hip": ["-ffp-contract=off"],
    "filter.hip": [],
    "solvers.hip": [],
    "lp.hip": [],
    "diff.hip": [],
    "batch.hip": [],
    "tiles.hip": [],
    "dcneg.hip": [],
    "rounding.hip": [],
    "separable.hip": [],
    "noalloc.hip": [],
    "abi.cpp": ["-x", "hip"],
    "workspace.cpp": ["-x", "hip"],
}


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    warn = [l for l in r.stderr.splitlines()
            if "warning" in l and "packed-fp32-ops" not in l]
    if warn:
        sys.stderr.write("\n".join(warn) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build()
