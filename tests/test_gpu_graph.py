"""pm_step under HIP graph capture: with no gradient recording and no
timing, a step is three kernel launches on the bound stream (no allocation,
no host synchronisation, no memset nodes), so a caller can capture it once
and replay it.  Every replay is checked against eager steps, with eager
library work and synchronisations between the replays."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm

from gpu_util import say

pytestmark = pytest.mark.gpu


def _problem(N, shape, seed):
    rng = np.random.default_rng(seed)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=((N + 1) ** 2,) + shape)
    return sa, ss, q, u


@pytest.mark.parametrize("prec", [0, 1])
def test_step_replayed_from_graph(prec):
    import torch
    N, shape, reps = 3, (4, 6, 64), 4
    nz, ny, nx = shape
    V = (N + 1) ** 2
    sa, ss, q, u = _problem(N, shape, 80 + prec)
    h, dt = 1 / 64, 0.5 / 64
    # eager reference after 1 .. reps steps
    pm.pm_set_precision(prec)
    pm.pm_init(N, nx, ny, nz, h, dt, sa, ss, q)
    try:
        for i in range(V):
            pm.pm_write(i, u[i])
        ref = []
        for _ in range(reps):
            pm.pm_step(1)
            ref.append(np.stack([pm.pm_read(i) for i in range(V)]))
    finally:
        pm.pm_finalize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    pm.pm_set_precision(prec)
    pm.pm_init(N, nx, ny, nz, h, dt, sa, ss, q)
    try:
        for i in range(V):
            pm.pm_write(i, u[i])
        pm.pm_bind_stream(stream.cuda_stream)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            pm.pm_step(1)
        # capture queued nothing: the state is still the initial one
        u0 = u[0] if prec == 0 else u[0].astype(np.float32).astype(np.float64)
        assert np.array_equal(pm.pm_read(0), u0)
        for k in range(reps):
            graph.replay()
            torch.cuda.synchronize()
            total = pm.pm_total()  # eager library work between replays
            got = np.stack([pm.pm_read(i) for i in range(V)])
            say("graph replay %d prec %d max diff %.3e" % (k, prec, np.abs(got - ref[k]).max()))
            assert np.array_equal(got, ref[k]), k
            assert abs(total - got[0].sum()) <= 1e-9 * np.abs(got[0]).sum()
    finally:
        pm.pm_bind_stream(None)
        pm.pm_finalize()
