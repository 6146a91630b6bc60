"""Build libipcomp.so (HIP for gfx950) in place.

Usage: python -m paper_2502_04093_amd.build   (or call build()).
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libipcomp.so")
# host-only C++ (no HIP API, no device code): compiled as plain C++
HOST_SOURCES = ["server.cpp", "schedule.cpp", "planner.cpp", "stream_format.cpp"]
# HIP: the runtime calls and the kernels
HIP_SOURCES = ["api.cpp", "kernels.hip", "level3.hip", "entropy.hip"]
SOURCES = HOST_SOURCES + HIP_SOURCES
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    out_tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           "-o", out_tmp, "-x", "c++"] + [os.path.join(CSRC, s) for s in HOST_SOURCES] + [
           "-x", "hip"] + [os.path.join(CSRC, s) for s in HIP_SOURCES] + [
           # ROCTx ranges around the library calls (rocprofv3 --marker-trace)
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
