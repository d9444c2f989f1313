"""A few steps of one bench workload through a given build of the library, for
rocprofv3 counter collection (measurement only).  The state is initialised as
bench.py does it (the workload's moments, written from the device).

    rocprofv3 --pmc FETCH_SIZE --kernel-include-regex k_sweep_win -o p -d DIR \\
        -- python3 bench_probe/sweep_counters.py --workload p39_large --prec fp64

A call pm_step(n) of the merged schedule launches n + 1 odd sweeps (the
first and the last ones half steps) and n even ones; the line printed at the
end gives the counts per parity over the two calls (warmup, then steps).
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lib", default=os.path.join(HERE, "libpm_counters.so"))
    ap.add_argument("--workload", default="p39_smooth")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--copy", action="store_true",
                    help="instead: libpm_probe.so's probes over 4 GiB buffers; its flat copies "
                         "(k_copy_flat, 4 GiB read and 4 GiB written each) calibrate the counters")
    a = ap.parse_args()
    if a.copy:
        import ctypes
        lib = ctypes.CDLL(os.path.join(HERE, "libpm_probe.so"))
        lib.pmp_ceilings.argtypes = [ctypes.c_longlong, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double)]
        out = (ctypes.c_double * 4)()
        rc = lib.pmp_ceilings(4 << 30, 256 * 1024, out)
        print(json.dumps({"copy_bytes": 4 << 30, "rc": rc, "gbs": list(out)}), flush=True)
        return 1 if rc else 0
    import torch
    import workloads
    from paper_2004_02833_amd import binding as pm
    pm.LIB_PATH = os.path.abspath(a.lib)
    w = workloads.RECIPES[a.workload]()
    dev = torch.device("cuda", 0)
    pm.pm_set_precision({"fp64": pm.PM_FP64, "fp32": pm.PM_FP32, "bf16": pm.PM_BF16}[a.prec])
    pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
    pm.pm_set_scattering(w.extra.get("scattering"))
    pm.pm_init(w.N, w.n, w.n, w.n, w.h, w.dt, w.sigma_a, w.sigma_s, w.q)
    pm.pm_set_scattering(None)
    for i in range(w.V):
        plane = w.moment_device(i, dev)
        pm.pm_write_dev(i, plane.data_ptr())
        del plane
    pm.pm_step(a.warmup)
    pm.pm_step(a.steps)
    pm.pm_sync()
    maxabs, nonfinite = pm.pm_check()
    pm.pm_finalize()
    print(json.dumps({"workload": w.name, "n": w.n, "N": w.N, "prec": a.prec, "lib": os.path.basename(a.lib),
                      "odd_sweeps": a.warmup + a.steps + 2, "even_sweeps": a.warmup + a.steps,
                      "maxabs": maxabs,
                      "nonfinite": nonfinite}), flush=True)
    return 1 if nonfinite else 0


if __name__ == "__main__":
    sys.exit(main())
