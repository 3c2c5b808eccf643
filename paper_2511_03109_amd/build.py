"""Build the native library libph.so in-tree (host C++ with g++/OpenMP, HIP for gfx950).

Usage: python -m paper_2511_03109_amd.build   (or call build()).
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libph.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["tree.cpp", "offline.cpp", "special.cpp", "tt.cpp"]
HIP_SOURCES = ["ph_api.hip", "k_instantiate.hip", "k_matvec.hip", "k_near_fused.hip", "k_coupling_bf16.hip", "k_hmatrix.hip", "k_offline.hip", "k_solve.hip"]
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
GXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose=False):
    """Compile every source and link libph.so (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(OBJ, src + ".o")
        _run(["g++", *GXX_FLAGS, "-I" + INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(OBJ, src + ".o")
        _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, "-I" + INCLUDE, "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-o", tmp, *objs, "-fopenmp", "-L" + os.path.join(ROCM, "lib"),
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
