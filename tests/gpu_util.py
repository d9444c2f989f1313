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


def window_index(shape, corner, B, R):
    """Periodic index arrays of the window [corner - R, corner + B + R) per axis."""
    return tuple((np.arange(-R, B + R) + corner[d]) % shape[d] for d in range(3))


def window_oracle(N, shape, h, dt, sa, ss, q, u_window, corner, B, R, nsteps):
    """FP64 oracle on a periodic window around a B^3 sub-block.  Every sweep
    reads one neighbour per direction, so after nsteps steps the error made by
    wrapping the window reaches at most 3 nsteps cells inward: with
    R >= 3 nsteps the central B^3 block equals the full-domain result."""
    from oracle import c_oracle
    assert R >= 3 * nsteps
    ix = window_index(shape, corner, B, R)
    sub = np.ix_(*ix)
    W = (B + 2 * R,) * 3
    qq = None if q is None else q[sub]
    out = c_oracle.run(N, W, h, dt, sa[sub], ss[sub], qq, u_window, nsteps)
    return out[:, R:R + B, R:R + B, R:R + B]


def progress(msg):
    """Progress line of a long GPU test, written when a piece of its work has
    ended: printed, and appended to gpurun_out/gpu_tests_progress.log so that
    a run whose output pytest captures still shows it advancing."""
    import os
    say(msg)
    d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    try:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "gpu_tests_progress.log"), "a") as f:
            f.write(msg + "\n")
    except OSError:
        pass


def oracle_run_chunked(N, shape, h, dt, sa, ss, q, u0, nsteps, chunk, label):
    """The C oracle over nsteps literal steps, run as pieces of `chunk` steps
    (the state is the only thing carried from one step to the next), with a
    progress line after each piece."""
    from oracle import c_oracle
    u = u0
    done = 0
    while done < nsteps:
        k = min(chunk, nsteps - done)
        u = c_oracle.run(N, shape, h, dt, sa, ss, q, u, k)
        done += k
        progress("%s: oracle %d/%d steps" % (label, done, nsteps))
    return u


class DegreeErrors:
    """Normwise error over all moments and per degree l: max |x - ref| over
    the moments of a degree divided by the largest |ref| of that degree."""

    def __init__(self, N):
        self.N = N
        self.num = np.zeros(N + 1)
        self.den = np.zeros(N + 1)

    def add(self, i, x, ref):
        l = int(np.floor(np.sqrt(i)))
        self.num[l] = max(self.num[l], float(np.abs(np.asarray(x) - ref).max()))
        self.den[l] = max(self.den[l], float(np.abs(ref).max()))

    def normwise(self):
        return float(self.num.max() / self.den.max())

    def per_degree(self):
        return self.num / np.where(self.den > 0, self.den, np.inf)
