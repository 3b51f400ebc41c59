"""Build libmfbcsr.so in-tree for gfx950 with hipcc.

Usage: python -m paper_1907_01005_amd.build  (or call build()).
Objects go to paper_1907_01005_amd/_build/, the library next to this file.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmfbcsr.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("MFB_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    p = os.path.join(ROCM, "bin", "hipcc")
    return p if os.path.exists(p) else (shutil.which("hipcc") or "hipcc")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
    # host planner: plain C++, geometric predicates must round as written
    planner_o = os.path.join(OUT, "planner.o")
    _run(["g++"] + common + ["-ffp-contract=off", "-c", os.path.join(CSRC, "planner.cpp"),
                             "-o", planner_o], verbose)
    # C boundary: host code that calls the HIP runtime
    capi_o = os.path.join(OUT, "capi.o")
    _run(["g++"] + common + ["-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
                             "-c", os.path.join(CSRC, "capi.cpp"), "-o", capi_o], verbose)
    # device kernels
    kern_o = os.path.join(OUT, "kernels.o")
    _run([hipcc] + common + [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                             "-packed-fp32-ops", "-munsafe-fp-atomics", "-c",
                             os.path.join(CSRC, "kernels.hip"), "-o", kern_o], verbose)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", planner_o, capi_o, kern_o,
          "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
