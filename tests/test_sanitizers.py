"""CPU builds of the host code under AddressSanitizer and UndefinedBehaviorSanitizer.

- The FP64 oracle (oracle/hmm_oracle.c) built by gcc with both sanitizers and
  -fno-sanitize-recover, loaded into a Python process that preloads gcc's ASan
  runtime, runs small workloads and special inputs and must match the ordinary
  build bit for bit (tests/sanitize/oracle_check.py).
- The host code of the C ABI (csrc/abi.hip: argument checks, workspace carve-up,
  tuning table, kernel resolution) built by hipcc with both sanitizers on the host
  side only, linked with the library's kernel objects into a driver that exercises
  every host path without a GPU (tests/sanitize/abi_host_check.cpp).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _run(["gcc", "-O2", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", lib, os.path.join(ROOT, "oracle", "hmm_oracle.c"), "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = _run([sys.executable, os.path.join(SAN, "oracle_check.py"), lib], env=env)
    assert "identical to the ordinary build" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_1310_3322_amd import build
    objdir = os.path.join(ROOT, "_build", "hip")
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in build.SOURCES if s != "abi.hip"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    # sanitizers on the host side only: every -fsanitize goes after -Xarch_host
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    abi = str(tmp_path / "abi_san.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "abi_host_check")
    _run([HIPCC, *build.FLAGS, "-g", "-O1", *san, "-c", os.path.join(build.CSRC, "abi.hip"), "-o", abi])
    _run([HIPCC, "-O1", "-g", "-std=c++17", *san, "-I", build.INCLUDE, "-c", os.path.join(SAN, "abi_host_check.cpp"),
          "-o", drv])
    # link with the LLVM driver that carries the sanitizer runtimes of the objects' compiler
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv, abi, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = _run([exe], env=env)
    assert "abi host checks passed" in r.stdout
