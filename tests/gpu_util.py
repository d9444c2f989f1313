"""Helpers for the GPU tests: run the HIP library through its C ABI."""
import sys

import numpy as np

import paper_2004_02833_amd as pm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(x, ref):
    """Normwise max-relative error max|x - ref| / max|ref|."""
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(ref).max())


def gpu_init(N, shape, h, dt, sa, ss, q=None, prec=0):
    nz, ny, nx = shape
    pm.pm_set_precision(prec)
    pm.pm_init(N, nx, ny, nz, h, dt, sa, ss, q)


def gpu_run(N, shape, h, dt, sa, ss, q, u0, nsteps, prec=0, moments=None):
    """u0: array (V, nz, ny, nx) or callable i -> plane.  Returns the moments."""
    V = (N + 1) ** 2
    gpu_init(N, shape, h, dt, sa, ss, q, prec)
    try:
        for i in range(V):
            pm.pm_write(i, u0(i) if callable(u0) else u0[i])
        pm.pm_step(nsteps)
        idx = range(V) if moments is None else moments
        return np.stack([pm.pm_read(i) for i in idx])
    finally:
        pm.pm_finalize()
