"""Benchmark of the staggered-grid P_N time step on one MI355X.

Workload: the P39 smooth-medium problem, 64^3 periodic cells, 1600 moments
(p39_smooth in workloads.py).  A step is one full Strang step (odd half step,
even full step, odd half step) over the whole grid, with the state resident in
HBM.  `value` runs them with the two odd half steps of consecutive steps
merged into one full odd step (2n+1 sweep launches for n steps); the literal
three-launch schedule is timed too ("three_sweep").  The metric is
GDoF-updates/s = cells * moments * steps / seconds / 1e9 (the paper's MLCUP/s
times 1e-3).

Prints ONE JSON line.  `value` is the FP64 path; the FP32 path is timed on
the same workload and reported in "fp32" together with its error against the
FP64 GPU run.  The roofline object is for the dominant kernel (the odd sweep,
launched twice per step): algorithmic bytes per launch over its mean launch
time from HIP events on the library's stream.  cpu_baseline times the FP64
CPU oracle on a bounded sample (a few steps of the same workload).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TABLE_BYTES = {1: 8 * 8, 0: 11 * 8}   # float64 table values read per cell: odd / even sweep
ESZ = {"f64": 8, "f32": 4, "bf16": 2}


def parity_counts(N):
    V = (N + 1) ** 2
    ve = sum(2 * l + 1 for l in range(0, N + 1, 2))
    return V, ve, V - ve


def sweep_bytes(N, ncell, esz, parity):
    """Algorithmic HBM bytes of one sweep launch: dual moments read once,
    target moments read and written once, plus the float64 tables."""
    V, ve, vo = parity_counts(N)
    tgt, dual = (vo, ve) if parity == 1 else (ve, vo)
    return ncell * ((dual + 2 * tgt) * esz + TABLE_BYTES[parity])


def kernel_source_hash():
    """Hash of the device sources with comments and whitespace removed, so
    that only code changes invalidate recorded counter data."""
    import re
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_02833_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            text = open(os.path.join(d, name)).read()
            text = re.sub(r"//[^\n]*", "", text)
            h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, dtype):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, or None
    when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        rec = data.get("%s/%s/%s" % (kernel, workload, dtype))
        if rec and rec.get("source_hash") == kernel_source_hash():
            return rec["bytes_per_launch"]
    except (ValueError, KeyError):
        pass
    return None


def sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except ImportError:
        pass


def run_gpu(pm, w, prec, steps, warmup, reps, keep_state=False):
    """Warmup, then exactly `steps` timed steps (the headline block, no
    per-sweep events), then `reps` more blocks of `steps` steps with HIP
    events around every sweep launch on the library's stream (the roofline:
    median over the blocks of the mean launch time), then one block with the
    literal three-sweep schedule."""
    import torch
    n = w.n
    dev = torch.device("cuda", 0)
    pm.pm_set_precision(prec)
    pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
    pm.pm_set_scattering(w.extra.get("scattering"))
    pm.pm_init(w.N, n, n, n, w.h, w.dt, w.sigma_a, w.sigma_s, w.q)
    pm.pm_set_scattering(None)
    try:
        for i in range(w.V):
            plane = w.moment_device(i, dev)
            pm.pm_write_dev(i, plane.data_ptr())
            del plane
        pm.pm_step(warmup)
        pm.pm_sync()
        sync()
        t0 = time.perf_counter()
        pm.pm_step(steps)
        pm.pm_sync()
        sync()
        t1 = time.perf_counter()
        blocks = []
        for _ in range(reps):
            pm.pm_timing(1)
            pm.pm_step(steps)
            blocks.append(pm.pm_sweep_times())
            pm.pm_timing(0)
        # the same steps with every step as its three substeps
        pm.pm_set_merge(0)
        t2 = time.perf_counter()
        pm.pm_step(steps)
        pm.pm_sync()
        sync()
        t3 = time.perf_counter()
        pm.pm_set_merge(1)
        state = None
        if keep_state:
            # sampled moments, and on very large grids every k-th cell of them
            buf = torch.empty(w.shape, dtype=torch.float64, device=dev)
            stride = max(1, w.n ** 3 // (1 << 22))
            state = []
            for i in state_moments(w):
                pm.pm_read_dev(i, buf.data_ptr())
                state.append(buf.reshape(-1)[::stride].cpu().numpy())
            del buf
        maxabs, nonfinite = pm.pm_check()
        return t1 - t0, blocks, t3 - t2, state, (maxabs, nonfinite)
    finally:
        pm.pm_finalize()
        pm.pm_bind_stream(0)


def copy_ceiling(gib):
    """Device-to-device copy of `gib` GiB with torch (one copy kernel per
    call): the practical HBM ceiling, and the reference dispatch whose PMC
    byte counters calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = int(gib * 2 ** 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / reps / 1e3
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * n * 4, "gbs": round(2 * n * 4 / sec / 1e9, 1)}


def degree_band_errors(w, state, ref_state):
    """Normwise error per band of degrees l (l = 0, then four equal bands),
    each relative to the largest reference value in its band."""
    idx = state_moments(w)
    deg = np.floor(np.sqrt(np.array(idx))).astype(int)
    edges = [0, 1] + [1 + (w.N * k + 3) // 4 for k in range(1, 4)] + [w.N + 1]
    out = {}
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = [j for j in range(len(idx)) if lo <= deg[j] < hi]
        if not sel:
            continue
        num = max(float(np.abs(state[j] - ref_state[j]).max()) for j in sel)
        den = max(float(np.abs(ref_state[j]).max()) for j in sel)
        out["l=%d" % lo if hi == lo + 1 else "l=%d-%d" % (lo, hi - 1)] = num / den if den > 0 else None
    return out


def state_moments(w):
    """Moments read back for the comparison between forms: all of them on
    grids up to ~1e9 values, an evenly spaced sample of 100 beyond (host
    memory; there every k-th cell is kept as well, see run_gpu)."""
    if w.n ** 3 * w.V <= 1_000_000_000:
        return list(range(w.V))
    return sorted(set(np.linspace(0, w.V - 1, 100).astype(int).tolist()))


def ceilings(ncell):
    """Measured bandwidth ceilings (libpm_probe.so): flat read, flat copy and
    a pure-memory kernel with the sweeps' access pattern, in GB/s."""
    import ctypes
    path = os.path.join(ROOT, "bench_probe", "libpm_probe.so")
    if not os.path.exists(path):
        from bench_probe import build as probe_build
        probe_build.build()
    lib = ctypes.CDLL(path)
    lib.pmp_ceilings.argtypes = [ctypes.c_longlong, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double)]
    out = (ctypes.c_double * 4)()
    rc = lib.pmp_ceilings(4 << 30, (ncell // 256) * 256, out)
    if rc != 0:
        return {"error": rc}
    return {"flat_read": round(out[0], 1), "flat_copy": round(out[1], 1),
            "sweep_pattern_f64": round(out[2], 1), "sweep_pattern_f32": round(out[3], 1),
            "unit": "GB/s"}


def step_bytes(N, esz):
    """Algorithmic bytes per DoF-update of one steady-state step for the
    literal schedule (two odd half-step sweeps and one even sweep) and the
    merged one that pm_step runs (one odd and one even sweep).  Bytes only:
    the bandwidth figure is the kernel's roofline."""
    V, ve, vo = parity_counts(N)
    three = ((4 * ve + 5 * vo) * esz + 2 * TABLE_BYTES[1] + TABLE_BYTES[0]) / V
    merged = ((3 * ve + 3 * vo) * esz + TABLE_BYTES[1] + TABLE_BYTES[0]) / V
    return {"bytes_per_dof_three_sweep": round(three, 3), "bytes_per_dof_merged": round(merged, 3)}


def roofline(N, ncell, esz, blocks):
    """The dominant kernel (the odd sweep): algorithmic bytes per launch over
    its launch time, the median over the timed blocks of each block's mean."""
    per = sorted(b["odd"][1] / max(b["odd"][0], 1) for b in blocks)
    per_even = sorted(b["even"][1] / max(b["even"][0], 1) for b in blocks)
    med = per[len(per) // 2] / 1e3
    byts = sweep_bytes(N, ncell, esz, 1)
    achieved = byts / med / 1e9
    ebytes = sweep_bytes(N, ncell, esz, 0)
    emed = per_even[len(per_even) // 2] / 1e3
    return {"kernel": "sweep_odd", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "bytes_per_launch": byts, "ms_per_launch": round(med * 1e3, 4),
            "ms_per_launch_blocks": [round(x, 4) for x in per], "launches_per_block": blocks[0]["odd"][0],
            "even_sweep": {"ms_per_launch": round(emed * 1e3, 4), "bytes_per_launch": ebytes,
                           "frac": round(ebytes / emed / 1e9 / HBM_PEAK_GBS, 4)}}


def adjoint_timing(pm):
    """Forward (recorded) and reverse pass of the gradient workload: P7,
    64^3, 200 steps, checkpoints every 20 steps, in FP64 and in FP32 storage;
    the FP32 gradients are compared with the FP64 ones (normwise)."""
    import torch
    import workloads
    w = workloads.p7_adjoint()
    dev = torch.device("cuda", 0)
    target = np.zeros(w.shape)
    out = {"workload": "%s: P%d, %d^3, %d steps, checkpoint every %d"
                       % (w.name, w.N, w.n, w.nsteps, w.checkpoint)}
    grads = {}
    for name, prec in (("fp64", pm.PM_FP64), ("fp32", pm.PM_FP32)):
        pm.pm_set_precision(prec)
        pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
        pm.pm_init(w.N, w.n, w.n, w.n, w.h, w.dt, w.sigma_a, w.sigma_s, w.q)
        try:
            for i in range(w.V):
                pm.pm_write(i, w.moment(i))
            pm.pm_set_checkpoint(w.checkpoint)
            pm.pm_sync()
            t0 = time.perf_counter()
            pm.pm_step(w.nsteps)
            pm.pm_sync()
            t1 = time.perf_counter()
            u0 = pm.pm_read(0)
            t2 = time.perf_counter()
            grads[name] = pm.pm_grad(u0 - target)
            t3 = time.perf_counter()
        finally:
            pm.pm_finalize()
            pm.pm_bind_stream(0)
        out[name] = {"forward_ms": round((t1 - t0) * 1e3, 2), "grad_ms": round((t3 - t2) * 1e3, 2)}
    for k, name in enumerate(("dsigma_a", "dsigma_s")):
        ref = grads["fp64"][k]
        out["fp32"]["rel_err_%s_vs_fp64" % name] = float(np.abs(grads["fp32"][k] - ref).max()
                                                        / np.abs(ref).max())
    # the FP64 numbers at the top level, as before
    out["forward_ms"], out["grad_ms"] = out["fp64"]["forward_ms"], out["fp64"]["grad_ms"]
    return out


def halo_timing(pm, N=39, prec_name="fp32", steps=5):
    """One GPU's share of the 160^3 P39 box split over 8 GPUs: the halo
    faces each sweep needs (pm_halo_pack into a staging buffer, then
    pm_halo_unpack from it; no transfer, one GPU) timed beside the sweeps of
    that share.  Two splits: 2 x 2 x 2 (80^3 sub-boxes, x faces included:
    one 4-byte value per 128-byte line there) and 1 x 2 x 4 (160 x 80 x 40:
    whole x rows, only y and z faces are exchanged)."""
    import torch
    import workloads
    PREC = {"fp64": (pm.PM_FP64, torch.float64, 8), "fp32": (pm.PM_FP32, torch.float32, 4)}
    prec, tdt, esz = PREC[prec_name]
    dev = torch.device("cuda", 0)
    out = {"moments": "P%d" % N, "dtype": prec_name, "unit": "ms"}
    for name, (nx, ny, nz), dirs in (("split_2x2x2", (80, 80, 80), 7), ("split_1x2x4", (160, 80, 40), 6)):
        rng = np.random.default_rng(1)
        shape = (nz, ny, nx)
        sa = 0.1 + 0.4 * rng.uniform(size=shape)
        ss = 1.0 - sa
        pm.pm_set_precision(prec)
        pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
        pm.pm_init(N, nx, ny, nz, 1.0 / 160, 0.5 / 160, sa, ss, None)
        try:
            buf = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev)
            for i in range((N + 1) ** 2):
                buf.normal_()
                pm.pm_write_dev(i, buf.data_ptr())
            del buf
            pm.pm_step(1)
            pm.pm_timing(1)
            pm.pm_step(steps)
            t = pm.pm_sweep_times()
            pm.pm_timing(0)
            sweep_ms = (t["odd"][1] / t["odd"][0] + t["even"][1] / t["even"][0])
            res = {"cells": nx * ny * nz, "shape_xyz": [nx, ny, nz],
                   "faces": "".join(a for d, a in enumerate("xyz") if (dirs >> d) & 1)}
            tot = 0.0
            for parity in (1, 0):
                n = pm.pm_halo_plan(N, nx, ny, nz, parity, dirs)
                stage = torch.empty(n, dtype=tdt, device=dev)
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                pm.pm_halo_pack(parity, stage.data_ptr(), dirs)       # warm
                pm.pm_halo_unpack(parity, stage.data_ptr(), dirs)
                ev[0].record()
                for _ in range(steps):
                    pm.pm_halo_pack(parity, stage.data_ptr(), dirs)
                ev[1].record()
                for _ in range(steps):
                    pm.pm_halo_unpack(parity, stage.data_ptr(), dirs)
                ev[2].record()
                torch.cuda.synchronize()
                pk = ev[0].elapsed_time(ev[1]) / steps
                un = ev[1].elapsed_time(ev[2]) / steps
                tot += pk + un
                res["odd_sweep" if parity else "even_sweep"] = {
                    "halo_elements": n, "halo_mb": round(n * esz / 1e6, 2),
                    "pack_ms": round(pk, 4), "unpack_ms": round(un, 4)}
                del stage
            res["sweeps_ms_per_step"] = round(sweep_ms, 4)
            res["halo_ms_per_step"] = round(tot, 4)
            res["halo_over_sweeps"] = round(tot / sweep_ms, 4)
            out[name] = res
        finally:
            pm.pm_finalize()
            pm.pm_bind_stream(0)
    return out


def cpu_baseline(w, steps, threads=0):
    """The C oracle on the host: every core (threads=0) or the given count."""
    from oracle import c_oracle
    c_oracle.build(force=False)
    u0 = w.initial()
    t0 = time.perf_counter()
    c_oracle.run(w.N, w.shape, w.h, w.dt, w.sigma_a, w.sigma_s, w.q, u0, steps, threads=threads,
                 scattering=w.extra.get("scattering"))
    dt = time.perf_counter() - t0
    threads = c_oracle.threads()
    return {"value": round(w.n ** 3 * w.V * steps / dt / 1e9, 5), "unit": "GDoF-updates/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d of %d steps of %s (P%d, %d^3), plain C/OpenMP FP64, %.1f s"
                      % (steps, w.nsteps, w.name, w.N, w.n, dt)}


def time_forms(pm, w, forms, args, say):
    """Time each storage form of workload w; the first form is the
    reference for the error of the others (sampled moments, normwise and per
    band of degrees)."""
    PREC = {"fp64": (pm.PM_FP64, 8, "f64"), "fp32": (pm.PM_FP32, 4, "f32"),
            "bf16": (pm.PM_BF16, 2, "bf16")}
    ncell, V = w.n ** 3, w.V
    results = {}
    ref_state = None
    for k, form in enumerate(forms):
        prec, esz, dname = PREC[form]
        say("bench: %s P%d %d^3, %s, %d warmup + %d steps, %d roofline blocks"
            % (w.name, w.N, w.n, form, args.warmup, args.steps, args.reps))
        keep = len(forms) > 1
        t, blocks, t3, state, chk = run_gpu(pm, w, prec, args.steps, args.warmup, args.reps,
                                            keep_state=keep)
        r = roofline(w.N, ncell, esz, blocks)
        r["traffic"] = measured_traffic("sweep_odd", w.name, dname)
        res = {"value": round(ncell * V * args.steps / t / 1e9, 3),
               "ms_per_step": round(t / args.steps * 1e3, 4),
               "three_sweep": {"value": round(ncell * V * args.steps / t3 / 1e9, 3),
                               "ms_per_step": round(t3 / args.steps * 1e3, 4)},
               "dtype": dname, "roofline": r, "step_bytes": step_bytes(w.N, esz),
               "state_check": {"max_abs": chk[0], "nonfinite": chk[1]}}
        if k == 0:
            ref_state = state
        elif state is not None and ref_state is not None:
            res["rel_err_vs_%s_gpu" % forms[0]] = (
                max(float(np.abs(a - b).max()) for a, b in zip(state, ref_state))
                / max(float(np.abs(b).max()) for b in ref_state))
            res["moments_compared"] = len(state)
            res["rel_err_by_degree"] = degree_band_errors(w, state, ref_state)
        results[form] = res
        del state
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=5,
                    help="timed blocks of --steps steps for the roofline (median)")
    ap.add_argument("--workload", default="p39_smooth")
    ap.add_argument("--large", default="p39_large",
                    help="second workload timed in the same line ('none' to skip)")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-steps-1thread", type=int, default=1,
                    help="steps of the one-thread oracle sample (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp64,fp32",
                    help="storage forms to time; the first is the headline value")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--bf16", action="store_true", help="also time the BF16-storage probe")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient timing")
    ap.add_argument("--no-halo", action="store_true", help="skip the halo pack/unpack timing")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the bandwidth ceilings (libpm_probe.so)")
    ap.add_argument("--copy-gib", type=float, default=4.0,
                    help="size of the calibration copy (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only: the step runs and is measured on a single MI355X; "
              "sharding the box across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.reps < 1:
        ap.error("--reps must be >= 1")

    import paper_2004_02833_amd as pm
    import workloads

    w = workloads.RECIPES[args.workload]()
    ncell = w.n ** 3
    V = w.V
    say = lambda *a: print(*a, file=sys.stderr, flush=True)

    copy = copy_ceiling(args.copy_gib) if args.copy_gib > 0 else None
    ceil = None if args.no_ceilings else ceilings(min(ncell, 262144))
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if args.no_fp32 and "fp32" in forms:
        forms.remove("fp32")
    if args.bf16 and "bf16" not in forms:
        forms.append("bf16")
    results = time_forms(pm, w, forms, args, say)
    head = results[forms[0]]

    large = None
    if args.large and args.large != "none" and args.large != args.workload:
        wl = workloads.RECIPES[args.large]()
        lres = time_forms(pm, wl, forms, args, say)
        large = {"workload": "%s: P%d (%d moments), %d^3 periodic cells, dx=1/%d, dt=dx/2"
                             % (wl.name, wl.N, wl.V, wl.n, wl.n),
                 "cells": wl.n ** 3, "moments": wl.V, "forms": lres}
        del wl

    halo = None
    if not args.no_halo:
        say("bench: halo faces of an 8-GPU split (one GPU's share)")
        halo = halo_timing(pm)

    adjoint = None
    if not args.no_adjoint:
        say("bench: adjoint timing")
        adjoint = adjoint_timing(pm)

    cpu = cpu1 = None
    if not args.no_cpu_baseline and w.n ** 3 * w.V > 1_000_000_000:
        say("bench: cpu oracle sample skipped for %s (host memory)" % w.name)
    elif not args.no_cpu_baseline:
        say("bench: cpu oracle sample (%d steps)" % args.cpu_steps)
        cpu = cpu_baseline(w, args.cpu_steps)
        if args.cpu_steps_1thread > 0:
            say("bench: cpu oracle sample on one thread (%d steps)" % args.cpu_steps_1thread)
            cpu1 = cpu_baseline(w, args.cpu_steps_1thread, threads=1)

    out = {
        "metric": "GDoF-updates/s (cell x moment per step) P39 3D; % HBM peak; FP32 vs FP64 error",
        "value": head["value"],
        "unit": "GDoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "schedule": "merged odd half steps: 2n+1 sweep launches per pm_step(n)",
        "three_sweep": head["three_sweep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": {"workload": "%s: P%d (%d moments), %d^3 periodic cells, dx=1/%d, dt=dx/2"
                               % (w.name, w.N, V, w.n, w.n),
                   "cells": ncell, "moments": V, "seed": w.seed},
        "roofline": head["roofline"],
        "step_bytes": head["step_bytes"],
        "forms": {f: r for f, r in results.items() if f != forms[0]},
        "large": large,
        "halo": halo,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "paper_context": "139.1 MLCUP/s = 0.139 GDoF-updates/s per core, P39 FP64, Haswell Xeon "
                         "E5-2623 v3 (kasper), optimised AVX2 sweeps; other machine, context only",
        "copy_ceiling": copy,
        "ceilings": ceil,
        "state_check": head["state_check"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
