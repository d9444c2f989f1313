"""Build libpm_probe.so, the bandwidth probes bench.py reports beside the
roofline (measurement only; not part of the P_N library).

    python -m bench_probe.build              # libpm_probe.so
    python -m bench_probe.build --counters   # libpm_counters.so

libpm_counters.so is the P_N library compiled from the product sources with
the product flags, except that a stub (scratch_stub.cpp) replaces the static
device scratch array of pm_check_noalloc: rocprofv3's counter collection
failed on the library while its code object held that device variable.  The
sweep kernels it runs are the product's.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpm_probe.so")
COUNTERS_LIB = os.path.join(HERE, "libpm_counters.so")


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-Wall", "-x", "hip",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-shared", "-o", tmp,
           os.path.join(HERE, "probe.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_counters(verbose=False):
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2004_02833_amd import build as pb
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    srcs = [(os.path.join(pb.CSRC, n), h) for n, h in pb.SOURCES if n != "scratch.hip"]
    srcs.append((os.path.join(HERE, "scratch_stub.cpp"), False))
    for src, is_hip in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = (["hipcc"] + pb.COMMON + ["-I" + pb.CSRC] + (["-x", "hip"] + pb.DEVFLAGS if is_hip else [])
               + ["-c", src, "-o", obj])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = COUNTERS_LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "-fPIC", "--offload-arch=" + pb.ARCH, "-o", tmp] + objs)
    os.replace(tmp, COUNTERS_LIB)
    return COUNTERS_LIB


if __name__ == "__main__":
    if "--counters" in sys.argv:
        print(build_counters(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
