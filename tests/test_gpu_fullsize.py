"""Full-size parity: the configurations run at their real grid sizes and in
the launch configuration bench.py times, checked on sampled 8^3 sub-blocks
against the FP64 oracle run on a periodic window around each block (exact by
the dependence radius, see test_window_oracle.py)."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm
import workloads

from gpu_util import relerr, say, window_index, window_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {pm.PM_FP64: 1e-12, pm.PM_FP32: 1e-5, pm.PM_BF16: 1e-2}
NAME = {pm.PM_FP64: "fp64", pm.PM_FP32: "fp32", pm.PM_BF16: "bf16"}


def run_blocks(w, prec, nsteps, corners, B, R, want_windows):
    """Run the library on the full grid; return the sub-blocks after nsteps
    and (optionally) the initial windows for the oracle."""
    dev = torch.device("cuda", 0)
    n = w.n
    pm.pm_set_precision(prec)
    pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
    pm.pm_init(w.N, n, n, n, w.h, w.dt, w.sigma_a, w.sigma_s, w.q)
    wins = None
    try:
        idx = [tuple(torch.as_tensor(a, device=dev) for a in window_index(w.shape, c, B, R))
               for c in corners]
        if want_windows:
            wins = [np.empty((w.V, B + 2 * R, B + 2 * R, B + 2 * R)) for _ in corners]
        for i in range(w.V):
            plane = w.moment_device(i, dev)
            pm.pm_write_dev(i, plane.data_ptr())
            if want_windows:
                for k, (iz, iy, ix) in enumerate(idx):
                    wins[k][i] = plane[iz][:, iy][:, :, ix].cpu().numpy()
            del plane
        pm.pm_step(nsteps)
        buf = torch.empty(w.shape, dtype=torch.float64, device=dev)
        blocks = [np.empty((w.V, B, B, B)) for _ in corners]
        for i in range(w.V):
            pm.pm_read_dev(i, buf.data_ptr())
            for k, c in enumerate(corners):
                iz, iy, ix = (torch.as_tensor((np.arange(B) + c[d]) % n, device=dev) for d in range(3))
                blocks[k][i] = buf[iz][:, iy][:, :, ix].cpu().numpy()
        m, bad = pm.pm_check()
        assert bad == 0
        return blocks, wins
    finally:
        pm.pm_finalize()
        pm.pm_bind_stream(0)


def check(w, precs, nsteps, corners, B=8):
    R = 3 * nsteps
    refs = None
    errs = {}
    for prec in precs:
        say("  %s %s %d^3, %d steps" % (w.name, NAME[prec], w.n, nsteps))
        blocks, wins = run_blocks(w, prec, nsteps, corners, B, R, refs is None)
        if refs is None:
            refs = [window_oracle(w.N, w.shape, w.h, w.dt, w.sigma_a, w.sigma_s, w.q, win, c, B, R,
                                  nsteps) for win, c in zip(wins, corners)]
            del wins
        errs[NAME[prec]] = max(relerr(b, r) for b, r in zip(blocks, refs))
        assert all(np.abs(r).max() > 0 for r in refs)
    say("  %s sub-block rel err %s" % (w.name, errs))
    for prec in precs:
        assert errs[NAME[prec]] <= TOL[prec], (NAME[prec], errs)


def test_p39_large_160_cubed():
    """P39 at 160^3 (6.6e9 unknowns; 52 GB in FP64, 26 GB in FP32, 13 GB in
    BF16), the grid whose rows are not multiples of 64 cells."""
    w = workloads.p39_large()
    rng = np.random.default_rng(11)
    corners = [tuple(int(v) for v in rng.integers(0, 160, 3)), (156, 0, 77)]
    check(w, (pm.PM_FP64, pm.PM_FP32, pm.PM_BF16), 2, corners)


def test_p7_lattice_128_cubed():
    """P7 absorber lattice at 128^3 (two 64-cell segments per row), 8 steps:
    blocks at the source block and across an absorber boundary."""
    w = workloads.p7_lattice()
    corners = [(58, 58, 58), (50, 60, 66)]
    check(w, (pm.PM_FP64, pm.PM_FP32), 8, corners)


def test_reactor_500_cubed_p19():
    """Reactor-vessel stand-in, P19 at 500^3 (5e10 unknowns: 200 GB in FP32,
    100 GB in BF16; rows of 500 cells use linear tiles): blocks across a rod
    lattice and the core edge."""
    w = workloads.reactor()
    n = w.n
    q = w.q
    # blocks centred on a rod cell: mid-core, and straddling the core's top face
    rods = np.nonzero(q[n // 2, :, n // 2 - 10:n // 2 + 10] > 0)
    y0, x0 = int(rods[0][len(rods[0]) // 2]), int(rods[1][0]) + n // 2 - 10
    ztop = int(np.nonzero(q[:, y0, x0] > 0)[0].max())
    corners = [(n // 2 - 4, y0 - 4, x0 - 4), (ztop - 3, y0 - 2, x0 - 5)]
    check(w, (pm.PM_FP32, pm.PM_BF16), 2, corners)


def test_p7_lattice_full_length_fp32_vs_fp64():
    """The P7 lattice configuration over its full 400 steps, where the oracle
    would need the whole domain: FP32 storage against the FP64 run (all 64
    moments, normwise, within the FP32 target), both finite; after one step
    from the zero state sum u_0 is exactly dt * sum q (no absorption on the
    source block)."""
    w = workloads.p7_lattice()
    n = w.n
    out = {}
    for prec in (pm.PM_FP64, pm.PM_FP32):
        say("  p7_lattice %s 128^3, %d steps" % (NAME[prec], w.nsteps))
        pm.pm_set_precision(prec)
        pm.pm_init(w.N, n, n, n, w.h, w.dt, w.sigma_a, w.sigma_s, w.q)
        try:
            pm.pm_step(1)
            total = pm.pm_total()
            tol = 1e-12 if prec == pm.PM_FP64 else 1e-6
            assert abs(total - w.dt * w.q.sum()) <= tol * w.dt * w.q.sum()
            pm.pm_step(w.nsteps - 1)
            mx, bad = pm.pm_check()
            assert bad == 0 and mx > 0
            out[prec] = np.stack([pm.pm_read(i) for i in range(w.V)])
        finally:
            pm.pm_finalize()
    e = relerr(out[pm.PM_FP32], out[pm.PM_FP64])
    say("  p7_lattice 400 steps: fp32 vs fp64 %.2e" % e)
    assert e <= 1e-5


def _full_length_forms(w, precs, moments):
    """Run w over its full step count in each storage form; return the
    normwise error of every other form against the first, over `moments`,
    computed on the device."""
    dev = torch.device("cuda", 0)
    n = w.n
    ref, err = None, {}
    buf = torch.empty(w.shape, dtype=torch.float64, device=dev)
    for prec in precs:
        say("  %s %s %d^3, %d steps" % (w.name, NAME[prec], n, w.nsteps))
        pm.pm_set_precision(prec)
        pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
        pm.pm_init(w.N, n, n, n, w.h, w.dt, w.sigma_a, w.sigma_s, w.q)
        try:
            for i in range(w.V):
                plane = w.moment_device(i, dev)
                pm.pm_write_dev(i, plane.data_ptr())
                del plane
            pm.pm_step(w.nsteps)
            mx, bad = pm.pm_check()
            assert bad == 0 and mx > 0
            if ref is None:
                ref = {}
                for i in moments:
                    pm.pm_read_dev(i, buf.data_ptr())
                    ref[i] = buf.clone()
                pm.pm_sync()
            else:
                num = den = 0.0
                for i in moments:
                    pm.pm_read_dev(i, buf.data_ptr())
                    num = max(num, float((buf - ref[i]).abs().max()))
                    den = max(den, float(ref[i].abs().max()))
                err[prec] = num / den
        finally:
            pm.pm_finalize()
            pm.pm_bind_stream(0)
    return err


def test_p39_smooth_full_length_forms():
    """P39 at 64^3 over its 100 steps: FP32 and BF16 storage against the FP64
    run over all 1600 moments (FP32 within its target; BF16 reported)."""
    w = workloads.p39_smooth()
    err = _full_length_forms(w, (pm.PM_FP64, pm.PM_FP32, pm.PM_BF16), range(w.V))
    say("  p39_smooth 100 steps: fp32 %.2e bf16 %.2e" % (err[pm.PM_FP32], err[pm.PM_BF16]))
    assert err[pm.PM_FP32] <= 1e-5
    assert err[pm.PM_BF16] <= 1e-1


def test_p39_large_full_length_forms():
    """P39 at 160^3 over its 50 steps: FP32 and BF16 storage against the FP64
    run on 100 evenly spaced moments."""
    w = workloads.p39_large()
    moments = sorted(set(np.linspace(0, w.V - 1, 100).astype(int).tolist()))
    err = _full_length_forms(w, (pm.PM_FP64, pm.PM_FP32, pm.PM_BF16), moments)
    say("  p39_large 50 steps: fp32 %.2e bf16 %.2e" % (err[pm.PM_FP32], err[pm.PM_BF16]))
    assert err[pm.PM_FP32] <= 1e-5
    assert err[pm.PM_BF16] <= 1e-1
