"""GPU parity with anisotropic scattering (per-degree coefficients
c_l = sigma_a + (1 - g_l) sigma_s, pm_set_scattering) against the FP64
oracle on the same seeded inputs: forward in FP64 / FP32 / BF16 storage,
both step schedules, exact decay and conservation, and the gradient."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm
from oracle import adjoint as adj
from oracle import c_oracle
from oracle import stepper as st

from gpu_util import gpu_run, relerr, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def oracle_built():
    c_oracle.build(force=False)
    yield
    pm.pm_finalize()


@pytest.fixture(autouse=True)
def isotropic_afterwards():
    yield
    pm.pm_finalize()
    pm.pm_set_scattering(None)
    pm.pm_set_merge(1)


def hg(a, N):
    """Henyey-Greenstein moments g_l = a^l, l = 1..N."""
    return [a ** l for l in range(1, N + 1)]


def problem(N, shape, seed):
    rng = np.random.default_rng(seed)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1.5, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=((N + 1) ** 2,) + tuple(shape))
    return rng, sa, ss, q, u


@pytest.mark.parametrize("N,shape", [(1, (3, 4, 5)), (3, (5, 6, 7)), (3, (2, 3, 70)),
                                     (7, (4, 6, 64)), (7, (3, 5, 12)), (8, (4, 4, 32)),
                                     (5, (3, 4, 160)), (4, (2, 3, 100))])
def test_small_and_ragged_fp64(N, shape):
    say("case aniso fp64", N, shape)
    rng, sa, ss, q, u = problem(N, shape, 100 + N)
    g = list(rng.uniform(-1, 1, N))
    h, dt = 0.2, 0.07
    ref = st.run(st.Setup(N, shape, h, dt, sa, ss, q, scattering=g), u, 5)
    pm.pm_set_scattering(g)
    got = gpu_run(N, shape, h, dt, sa, ss, q, u, 5)
    e = relerr(got, ref)
    say("  err %.2e" % e)
    assert e <= FP64_TOL


@pytest.mark.parametrize("merge", [0, 1])
def test_schedules_and_checkpoints(merge):
    """Three-sweep and merged schedules, also split at checkpoints."""
    N, shape, n = 7, (5, 6, 16), 9
    say("case aniso schedule", merge)
    _, sa, ss, q, u = problem(N, shape, 110)
    g = hg(0.7, N)
    h, dt = 0.15, 0.05
    ref = st.run(st.Setup(N, shape, h, dt, sa, ss, q, scattering=g), u, n)
    pm.pm_set_merge(merge)
    pm.pm_set_scattering(g)
    for ck in (0, 4):
        pm.pm_set_precision(pm.PM_FP64)
        pm.pm_init(N, shape[2], shape[1], shape[0], h, dt, sa, ss, q)
        for i in range(64):
            pm.pm_write(i, u[i])
        if ck:
            pm.pm_set_checkpoint(ck)
        pm.pm_step(n)
        got = np.stack([pm.pm_read(i) for i in range(64)])
        pm.pm_finalize()
        assert relerr(got, ref) <= 1e-13, ck


def test_p39_fp64_fp32_bf16():
    """P39 with Henyey-Greenstein moments (a = 0.8) on 20 x 24 x 32 cells
    against the C oracle."""
    N, shape, n = 39, (20, 24, 32), 2
    say("case aniso P39", shape)
    _, sa, ss, q, _ = problem(1, shape, 120)
    rng = np.random.default_rng(121)
    V = (N + 1) ** 2
    u = rng.normal(scale=1e-3, size=(V,) + shape)
    u[0] += 1.0
    g = hg(0.8, N)
    h, dt = 1 / 32, 0.5 / 32
    ref = c_oracle.run(N, shape, h, dt, sa, ss, q, u, n, scattering=g)
    for prec, tol in ((pm.PM_FP64, FP64_TOL), (pm.PM_FP32, FP32_TOL), (pm.PM_BF16, 2e-2)):
        pm.pm_set_scattering(g)
        got = gpu_run(N, shape, h, dt, sa, ss, q, u, n, prec=prec)
        e = relerr(got, ref)
        say("  prec %d err %.2e" % (prec, e))
        assert e <= tol, prec


@pytest.mark.parametrize("shape", [(4, 6, 64), (3, 5, 12), (2, 3, 7), (3, 4, 160), (2, 3, 100), (3, 4, 128)])
def test_fp32_bf16_small_shapes(shape):
    N = 5
    _, sa, ss, q, u = problem(N, shape, 130)
    g = hg(-0.5, N)
    h, dt = 0.2, 0.07
    ref = st.run(st.Setup(N, shape, h, dt, sa, ss, q, scattering=g), u, 4)
    pm.pm_set_scattering(g)
    e32 = relerr(gpu_run(N, shape, h, dt, sa, ss, q, u, 4, prec=pm.PM_FP32), ref)
    pm.pm_set_scattering(g)
    e16 = relerr(gpu_run(N, shape, h, dt, sa, ss, q, u, 4, prec=pm.PM_BF16), ref)
    say("aniso small %s fp32 %.2e bf16 %.2e" % (shape, e32, e16))
    assert e32 <= FP32_TOL
    assert e16 <= 2e-2


def test_exact_decay_and_conservation_on_gpu():
    """Homogeneous state and medium: moment (l, m) decays as exp(-c_l t);
    sigma_a = 0: sum u_0 is conserved."""
    N, shape = 4, (4, 4, 8)
    sa, ss = 0.3, 1.2
    g = [0.5, -0.25, 0.125, 0.9]
    c = np.array([sa] + [sa + (1 - v) * ss for v in g])
    V = (N + 1) ** 2
    ell = np.array([int(np.floor(np.sqrt(i))) for i in range(V)])
    u0 = np.arange(1.0, V + 1.0)[:, None, None, None] * np.ones((V,) + shape)
    h, dt, n = 0.1, 0.04, 6
    pm.pm_set_scattering(g)
    got = gpu_run(N, shape, h, dt, np.full(shape, sa), np.full(shape, ss), None, u0, n)
    want = u0[:, 0, 0, 0] * np.exp(-c[ell] * n * dt)
    assert np.abs(got[:, 0, 0, 0] - want).max() <= 1e-13 * V
    assert np.abs(got - got[:, :1, :1, :1]).max() <= 1e-15 * V
    rng = np.random.default_rng(140)
    u = rng.normal(size=(V,) + shape)
    pm.pm_set_precision(pm.PM_FP64)
    pm.pm_init(N, shape[2], shape[1], shape[0], h, dt, np.zeros(shape), rng.uniform(0, 2, shape))
    for i in range(V):
        pm.pm_write(i, u[i])
    pm.pm_step(10)
    assert abs(pm.pm_total() - u[0].sum()) <= 1e-13 * np.abs(u[0]).sum()


def test_reset_to_isotropic():
    """pm_set_scattering(None) restores the isotropic path exactly."""
    N, shape = 3, (4, 5, 6)
    _, sa, ss, q, u = problem(N, shape, 150)
    iso = gpu_run(N, shape, 0.2, 0.07, sa, ss, q, u, 3)
    pm.pm_set_scattering([0.5, 0.2])
    aniso = gpu_run(N, shape, 0.2, 0.07, sa, ss, q, u, 3)
    pm.pm_set_scattering(None)
    again = gpu_run(N, shape, 0.2, 0.07, sa, ss, q, u, 3)
    assert np.array_equal(iso, again)
    assert relerr(aniso, iso) > 1e-6


@pytest.mark.parametrize("N,shape,nsteps,ck", [(3, (4, 5, 6), 5, 2), (2, (1, 2, 9), 4, 4),
                                               (5, (3, 4, 64), 3, 1)])
def test_grad_matches_oracle(N, shape, nsteps, ck):
    say("case aniso adjoint", N, shape)
    rng, sa, ss, q, u = problem(N, shape, 160 + N)
    g = list(rng.uniform(-0.9, 0.9, N))
    tgt = rng.normal(size=shape)
    h, dt = 0.2, 0.07
    L, ga, gs, _ = adj.loss_and_grad(st.Setup(N, shape, h, dt, sa, ss, q, scattering=g), u, nsteps, tgt)
    for prec, tol in ((pm.PM_FP64, 1e-12), (pm.PM_FP32, 1e-4)):
        pm.pm_set_scattering(g)
        pm.pm_set_precision(prec)
        pm.pm_init(N, shape[2], shape[1], shape[0], h, dt, sa, ss, q)
        try:
            for i in range((N + 1) ** 2):
                pm.pm_write(i, u[i])
            pm.pm_set_checkpoint(ck)
            pm.pm_step(nsteps)
            u0T = pm.pm_read(0)
            dsa, dss = pm.pm_grad(u0T - tgt)
        finally:
            pm.pm_finalize()
        ea, es = relerr(dsa, ga), relerr(dss, gs)
        say("  prec %d grad err %.2e %.2e" % (prec, ea, es))
        assert ea <= tol and es <= tol, prec
