"""The byte models of bench.py (no GPU): the per-launch sweep bytes, the two
per-step models, and the moment counts they use, checked against each other
and against the P39 counts (V = 1600, 780 even and 820 odd moments)."""
import bench


def test_parity_counts_p39():
    assert bench.parity_counts(39) == (1600, 780, 820)
    assert bench.parity_counts(3) == (16, 6, 10)
    assert bench.parity_counts(7) == (64, 28, 36)


def test_odd_sweep_bytes_p39_64():
    # dual (even) planes read once, odd planes read and written, 8 table values
    ncell = 64 ** 3
    assert bench.sweep_bytes(39, ncell, 8, 1) == ncell * ((780 + 2 * 820) * 8 + 64)
    assert bench.sweep_bytes(39, ncell, 8, 1) == 5091885056
    assert bench.sweep_bytes(39, ncell, 4, 0) == ncell * ((820 + 2 * 780) * 4 + 88)


def test_step_bytes_are_sums_of_sweeps():
    for N in (3, 7, 39):
        V = bench.parity_counts(N)[0]
        for esz in (8, 4, 2):
            odd = bench.sweep_bytes(N, 1, esz, 1)
            even = bench.sweep_bytes(N, 1, esz, 0)
            m = bench.step_bytes(N, esz)
            assert abs(m["bytes_per_dof_three_sweep"] - (2 * odd + even) / V) < 1e-3
            assert abs(m["bytes_per_dof_merged"] - (odd + even) / V) < 1e-3
            assert set(m) == {"bytes_per_dof_three_sweep", "bytes_per_dof_merged"}


def test_step_bytes_p39():
    assert abs(bench.step_bytes(39, 8)["bytes_per_dof_three_sweep"] - 36.235) < 1e-3
    assert abs(bench.step_bytes(39, 4)["bytes_per_dof_three_sweep"] - 18.185) < 1e-3


def test_roofline_takes_the_median_block():
    blocks = [{"odd": (21, 21 * t), "even": (20, 20 * 0.9 * t)} for t in (1.2, 1.0, 1.1, 5.0, 1.05)]
    r = bench.roofline(39, 64 ** 3, 8, blocks)
    assert r["ms_per_launch"] == 1.1
    assert abs(r["achieved"] - 5091885056 / 1.1e-3 / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000) < 1e-4
    assert r["even_sweep"]["ms_per_launch"] == 0.99


def test_source_hash_ignores_comments_not_code(tmp_path, monkeypatch):
    """Recorded traffic counters stay valid across comment and whitespace
    edits of the device sources and are invalidated by code edits."""
    import os
    import shutil
    src = os.path.join(bench.ROOT, "paper_2004_02833_amd", "csrc")
    dst = tmp_path / "paper_2004_02833_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    k = dst / "kernels.hip"
    text = k.read_text()
    k.write_text(text.replace("namespace pm {", "namespace pm {  // a comment\n\n", 1))
    assert bench.kernel_source_hash() == h0
    k.write_text(text.replace("namespace pm {", "namespace pm {\nconstexpr int kUnused = 1;", 1))
    assert bench.kernel_source_hash() != h0
    k.write_text(text)
    assert bench.kernel_source_hash() == h0


def test_traffic_summary_scales_and_splits_by_parity(tmp_path):
    """bench_probe/traffic_summary.py: counters scaled by the copy's known
    bytes, odd and even launches told apart by their writes, bytes per launch
    keyed by the source hash bench.py checks."""
    import json
    from bench_probe import traffic_summary as ts

    def write(name, counter, vals):
        d = tmp_path / name
        d.mkdir()
        with open(d / "p_counter_collection.csv", "w") as f:
            f.write("Dispatch_Id,Counter_Name,Counter_Value\n")
            for i, v in enumerate(vals):
                f.write("%d,%s,%r\n" % (i, counter, v))

    kib = 4 * 2 ** 30 / 1024
    write("copy_FETCH_SIZE", "FETCH_SIZE", [kib / 2] * 3)   # reads 2x what FETCH_SIZE shows
    write("copy_WRITE_SIZE", "WRITE_SIZE", [kib] * 3)
    ncell = 64 ** 3
    odd, even = bench.sweep_bytes(39, ncell, 8, 1), bench.sweep_bytes(39, ncell, 8, 0)
    w_odd, w_even = 820 * 8 * ncell, 780 * 8 * ncell
    # launches odd, even, odd; fetched bytes 1.2x the algorithmic reads
    f = [1.2 * (odd - w_odd) / 2048, 1.2 * (even - w_even) / 2048, 1.2 * (odd - w_odd) / 2048]
    write("p39_smooth_fp64_FETCH_SIZE", "FETCH_SIZE", f)
    write("p39_smooth_fp64_WRITE_SIZE", "WRITE_SIZE", [w_odd / 1024, w_even / 1024, w_odd / 1024])
    out = tmp_path / "traffic.json"
    ts.main(str(tmp_path), str(out))
    rec = json.load(open(out))
    assert set(rec) == {"sweep_odd/p39_smooth/f64", "sweep_even/p39_smooth/f64"}
    assert rec["sweep_odd/p39_smooth/f64"]["source_hash"] == bench.kernel_source_hash()
    got = rec["sweep_odd/p39_smooth/f64"]["bytes_per_launch"]
    assert abs(got - (1.2 * (odd - w_odd) + w_odd)) < 16
    got = rec["sweep_even/p39_smooth/f64"]["bytes_per_launch"]
    assert abs(got - (1.2 * (even - w_even) + w_even)) < 16
