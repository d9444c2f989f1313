"""Traffic of the sweep kernels from rocprofv3 counter runs (measurement only).

    python3 bench_probe/traffic_summary.py DIR

DIR holds one rocprofv3 output directory per run, named
    copy_<COUNTER>                           (calibration: libpm_probe's flat copy of 4 GiB)
    <workload>_<prec>_<COUNTER>              (bench_probe/sweep_counters.py)
with COUNTER FETCH_SIZE or WRITE_SIZE and the CSV written as p_counter_collection.csv
(rocprofv3 ... --output-format csv -o p).  Each counter is scaled by the factor
that makes the copy's reading equal its known bytes; odd and even sweeps are
told apart by their writes (820 against 780 planes at P39).  Writes
profiles/traffic.json (bytes per launch, keyed by the hash of the device
sources that bench.py checks) and prints a Markdown table.
"""
import csv
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

COPY_BYTES = 4 << 30  # read (FETCH_SIZE) and written (WRITE_SIZE) per copy
SIZES = {"p39_smooth": 64, "p39_large": 160, "p39_aniso": 64}
ESZ = {"fp64": 8, "fp32": 4, "bf16": 2}


def values(path):
    rows = list(csv.DictReader(open(os.path.join(path, "p_counter_collection.csv"))))
    return [float(r["Counter_Value"]) for r in rows]


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


def main(root, out_path=None):
    import bench
    ff = COPY_BYTES / (median(values(os.path.join(root, "copy_FETCH_SIZE"))) * 1024)
    wf = COPY_BYTES / (median(values(os.path.join(root, "copy_WRITE_SIZE"))) * 1024)
    V, ve, vo = bench.parity_counts(39)
    out, lines = {}, []
    for wl, n in SIZES.items():
        for prec, esz in ESZ.items():
            fdir = os.path.join(root, "%s_%s_FETCH_SIZE" % (wl, prec))
            wdir = os.path.join(root, "%s_%s_WRITE_SIZE" % (wl, prec))
            if not (os.path.isdir(fdir) and os.path.isdir(wdir)):
                continue
            f, w = values(fdir), values(wdir)
            if len(f) != len(w):
                raise SystemExit("%s %s: %d FETCH_SIZE and %d WRITE_SIZE dispatches" % (wl, prec, len(f), len(w)))
            mid = 0.5 * (max(w) + min(w))
            for parity, name in ((1, "sweep_odd"), (0, "sweep_even")):
                sel = [i for i in range(len(w)) if (w[i] > mid) == (parity == 1)]
                fb = sum(f[i] for i in sel) / len(sel) * 1024 * ff
                wb = sum(w[i] for i in sel) / len(sel) * 1024 * wf
                alg = bench.sweep_bytes(39, n ** 3, esz, parity)
                key = "%s/%s/%s" % (name, wl, {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec])
                out[key] = {"bytes_per_launch": int(round(fb + wb)), "source_hash": bench.kernel_source_hash()}
                lines.append("| %s | %s | %s | %d | %.4g | %.4g | %.4g | %.3f |" % (
                    wl, prec, name, len(sel), fb, wb, alg, (fb + wb) / alg))
    path = out_path or os.path.join(ROOT, "profiles", "traffic.json")
    json.dump(dict(sorted(out.items())), open(path, "w"), indent=1)
    print("calibration (flat copy of %d bytes): FETCH_SIZE x %.4f KiB, WRITE_SIZE x %.4f KiB" % (COPY_BYTES, ff, wf))
    print("| workload | form | kernel | launches | fetched B | written B | algorithmic B | ratio |")
    print("|---|---|---|---|---|---|---|---|")
    print("\n".join(lines))
    return out


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else None)
