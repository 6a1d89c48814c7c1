"""Compiles the HIP sources of libhmm_mi355x.so for gfx950 (in-tree).

    python -m paper_1310_3322_amd.build        # or __graft_entry__.build()
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhmm_mi355x.so")
# the same sources with the kernels' bounds checks compiled in (-DHMM_DEBUG)
LIB_DEBUG = os.path.join(PKG, "libhmm_mi355x_debug.so")
OBJDIR = os.path.join(ROOT, "_build", "hip")

SOURCES = ["planner.hip", "fwd_plain.hip", "fwd_mfma.hip", "fwd_mfma32.hip", "fwd_coop.hip", "fwd_scan.hip", "adj_mfma.hip", "adj_coop.hip", "viterbi.hip", "abi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 VALU instructions are disabled for all device code.  MFMA
# accumulators are allocated in ordinary VGPRs (not AGPRs), which saves the
# copies between the two files in the per-step epilogues.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form", "-I", INCLUDE]


def _compile(src: str, debug: bool = False) -> str:
    objdir = OBJDIR + ("_debug" if debug else "")
    obj = os.path.join(objdir, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *(["-DHMM_DEBUG"] if debug else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, debug: bool = False) -> str:
    """Builds libhmm_mi355x.so, or with debug=True libhmm_mi355x_debug.so (bounds checks in the kernels)."""
    lib = LIB_DEBUG if debug else LIB
    os.makedirs(OBJDIR + ("_debug" if debug else ""), exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, debug), SOURCES))
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    if "--debug" in sys.argv[1:]:
        build(verbose=True, debug=True)
    sys.exit(0)
