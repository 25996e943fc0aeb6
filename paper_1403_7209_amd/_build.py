"""Builds libopflux.so in place: host planner (g++), API and kernels (hipcc, gfx950)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libopflux.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# Packed FP32 instructions are switched off for every HIP translation unit.
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{INC}"]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-pthread", "-Wall", "-Wextra", f"-I{INC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objs = []
    o = os.path.join(BUILD, "planner.o")
    _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "planner.cpp"), "-o", o], verbose)
    objs.append(o)
    for src in ("opflux.cpp", "kernels.hip", "geometry.hip"):
        o = os.path.join(BUILD, src.split(".")[0] + ".o")
        _run([hipcc, *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
          f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64", "-pthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
