"""Build the PCV HIP library (libpcv.so) in-tree for gfx950.

Usage: python -m paper_2310_07002_amd.build   (or call build()).
Each source is compiled to an object with hipcc, then linked into one shared
library next to this file.  Compilation needs no GPU.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpcv.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# (source, extra flags, object name).  The VALU kernels are templates over
# the arithmetic type and the family; k_valu.hip is compiled once per pair
# (each instance emits one pair's kernels) and once more for the dispatchers,
# so the long device compilations run in parallel.
_VALU_INST = [("k_valu.hip", [f"-DPCV_VALU_T={t}", f"-DPCV_VALU_FAM={fam}"], f"k_valu_{t}_{fam}.o")
              for t in ("double", "float") for fam in range(5)]
SOURCES = [("api.hip", [], "api.o"), ("k_common.hip", [], "k_common.o"), ("k_valu.hip", [], "k_valu.o"),
           ("k_mfma.hip", [], "k_mfma.o"), ("posthoc.hip", [], "posthoc.o"),
           ("calib.hip", [], "calib.o")] + _VALU_INST
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed fp32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _compile(job) -> str:
    src, extra, name = job
    obj = os.path.join(BUILD_DIR, name)
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + src + " " + " ".join(extra))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), os.cpu_count() or 4, 16))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
