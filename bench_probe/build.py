"""Build libpm_probe.so, the bandwidth probes bench.py reports beside the
roofline (measurement only; not part of the P_N library).

    python -m bench_probe.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpm_probe.so")


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


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
