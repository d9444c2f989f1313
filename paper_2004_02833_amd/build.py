"""Build libpm.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2004_02833_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpm.so")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code.
DEVFLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH, "-Wall",
          "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]
SOURCES = [("api.cpp", False), ("flux.cpp", False), ("kernels.hip", True), ("scratch.hip", True)]


def build(verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for name, is_hip in SOURCES:
        src = os.path.join(CSRC, name)
        obj = os.path.join(objdir, name + ".o")
        cmd = ["hipcc"] + COMMON + (["-x", "hip"] + DEVFLAGS if is_hip else []) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
