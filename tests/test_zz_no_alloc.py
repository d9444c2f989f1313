"""The allocation-free variant of pm_check (pm_check_noalloc): partial
results in the library's static device scratch, outputs written to caller
device pointers.  Checked against pm_check on two calls in a row, the
second on a smaller grid, with non-finite values present in one of them."""
import ctypes

import numpy as np
import pytest

import paper_2004_02833_amd as pm

from gpu_util import gpu_init, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def check_both(case):
    dev = torch.device("cuda", 0)
    out_max = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    out_cnt = torch.full((1,), -1, dtype=torch.int64, device=dev)
    pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
    pm.pm_check_noalloc(out_max.data_ptr(), out_cnt.data_ptr())
    torch.cuda.synchronize()
    m_ref, k_ref = pm.pm_check()
    m, k = float(out_max.item()), int(out_cnt.item())
    say("  %s: noalloc (%r, %d) pm_check (%r, %d)" % (case, m, k, m_ref, k_ref))
    assert k == k_ref
    assert m == m_ref


def test_check_noalloc_matches_pm_check():
    rng = np.random.default_rng(17)
    try:
        # a large grid first: P7 on 96 x 80 x 64 cells, two NaNs and an infinity
        shape = (64, 80, 96)
        gpu_init(7, shape, 0.01, 0.004, rng.uniform(0, 1, shape), rng.uniform(0, 1, shape))
        for i in range(64):
            pm.pm_write(i, rng.normal(size=shape))
        bad = rng.normal(size=shape)
        bad[3, 4, 5] = np.nan
        bad[60, 70, 80] = np.inf
        bad[0, 0, 0] = -np.nan
        pm.pm_write(17, bad)
        check_both("P7 96x80x64 with non-finite values")
        pm.pm_finalize()
        # then a smaller one, all finite: stale partials of the first call must not leak
        shape = (5, 3, 7)
        gpu_init(3, shape, 0.2, 0.05, rng.uniform(0, 1, shape), rng.uniform(0, 1, shape), prec=pm.PM_FP32)
        for i in range(16):
            pm.pm_write(i, rng.normal(size=shape))
        pm.pm_step(2)
        check_both("P3 7x3x5 FP32, finite")
    finally:
        pm.pm_finalize()
        pm.pm_bind_stream(0)


def test_check_noalloc_errors():
    pm.pm_finalize()
    assert pm.lib().pm_check_noalloc(ctypes.c_void_p(8), ctypes.c_void_p(8)) == pm.PM_ESTATE
    gpu_init(1, (2, 2, 2), 0.5, 0.1, np.zeros((2, 2, 2)), np.zeros((2, 2, 2)))
    try:
        assert pm.lib().pm_check_noalloc(None, None) == pm.PM_EINVAL
    finally:
        pm.pm_finalize()
