"""Builds libchromstrip.so (host enumerator + gfx950 HIP kernels + C ABI).

    python -m paper_1005_3609_amd.build        # or paper_1005_3609_amd.build.build()

Always recompiles.  Objects go to paper_1005_3609_amd/_build/, the library
to paper_1005_3609_amd/libchromstrip.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libchromstrip.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# Packed-fp32 instructions stay off in every HIP compile.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = [
        (["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "states.cpp"), "-o",
          os.path.join(OUT_DIR, "states.o")]),
        (["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "maps.cpp"), "-o",
          os.path.join(OUT_DIR, "maps.o")]),
        ([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "runtime.hip"), "-o",
          os.path.join(OUT_DIR, "runtime.o")]),
    ]
    with ThreadPoolExecutor(4) as ex:
        logs = list(ex.map(_run, jobs))
    tmp = LIB + ".tmp"
    logs.append(_run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp,
                      os.path.join(OUT_DIR, "states.o"), os.path.join(OUT_DIR, "maps.o"),
                      os.path.join(OUT_DIR, "runtime.o"), "-lpthread"]))
    os.replace(tmp, LIB)
    if verbose:
        for log in logs:
            if log.strip():
                print(log, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
