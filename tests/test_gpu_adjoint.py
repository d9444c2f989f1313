"""GPU adjoint: pm_grad (transposed steps from checkpoints) against the FP64
oracle adjoint, and against central finite differences of the GPU forward."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm
from oracle import adjoint as adj
from oracle import c_oracle
from oracle import stepper as st

from gpu_util import gpu_init, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def oracle_built():
    c_oracle.build(force=False)
    yield
    pm.pm_finalize()


def gpu_grad(N, shape, h, dt, sa, ss, q, u0, nsteps, ck, target, prec=0):
    gpu_init(N, shape, h, dt, sa, ss, q, prec)
    try:
        for i in range((N + 1) ** 2):
            pm.pm_write(i, u0[i])
        pm.pm_set_checkpoint(ck)
        pm.pm_step(nsteps)
        u0T = pm.pm_read(0)
        dsa, dss = pm.pm_grad(u0T - target)
        u0T_after = pm.pm_read(0)
        assert np.array_equal(u0T, u0T_after), "pm_grad must leave the forward state unchanged"
        L = 0.5 * float(np.sum((u0T - target) ** 2))
        return L, dsa, dss
    finally:
        pm.pm_finalize()


# rows of 64 cells run the transposed sweeps on whole-row waves (x
# neighbours by lane rotation, a barrier per column; nz = 5 leaves waves past
# the grid in the last tile)
@pytest.mark.parametrize("N,shape,nsteps,ck", [(3, (4, 5, 6), 7, 3), (1, (3, 3, 3), 4, 1),
                                               (2, (1, 2, 9), 5, 5), (3, (2, 3, 70), 3, 2),
                                               (3, (3, 2, 64), 4, 2), (5, (5, 3, 64), 3, 3),
                                               # chunk tiles (rows longer than 64 cells)
                                               (3, (2, 2, 96), 4, 2), (2, (1, 64, 65), 3, 2)])
def test_grad_matches_numpy_oracle(N, shape, nsteps, ck):
    say("case adjoint small", N, shape, nsteps, ck)
    rng = np.random.default_rng(N * 7 + nsteps)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=((N + 1) ** 2,) + shape)
    tgt = rng.normal(size=shape)
    h, dt = 0.2, 0.07
    L, ga, gs, _ = adj.loss_and_grad(st.Setup(N, shape, h, dt, sa, ss, q), u, nsteps, tgt)
    L2, ga2, gs2 = gpu_grad(N, shape, h, dt, sa, ss, q, u, nsteps, ck, tgt)
    assert abs(L - L2) <= 1e-13 * L
    assert relerr(ga2, ga) <= 1e-12
    assert relerr(gs2, gs) <= 1e-12


def test_grad_p7_reduced_vs_c_oracle():
    """The gradient workload recipe (P7, blocks of 4^3) at 16^3, 40 steps,
    checkpoints every 20 steps, against the C oracle adjoint."""
    import workloads
    w = workloads.p7_adjoint(n=16, nsteps=40)
    say("case adjoint p7 16^3")
    u0 = w.initial()
    tgt = c_oracle.run(w.N, w.shape, w.h, w.dt, w.extra["perturbed_sigma_a"], w.sigma_s, w.q,
                       u0, w.nsteps)[0]
    L, ga, gs = c_oracle.grad(w.N, w.shape, w.h, w.dt, w.sigma_a, w.sigma_s, w.q, u0, w.nsteps,
                              w.checkpoint, tgt)
    L2, ga2, gs2 = gpu_grad(w.N, w.shape, w.h, w.dt, w.sigma_a, w.sigma_s, w.q, u0, w.nsteps,
                            w.checkpoint, tgt)
    say("p7 16^3 adjoint rel err", relerr(ga2, ga), relerr(gs2, gs))
    assert abs(L - L2) <= 1e-12 * L
    assert relerr(ga2, ga) <= 1e-11
    assert relerr(gs2, gs) <= 1e-11


@pytest.mark.parametrize("N,shape,nsteps,ck", [(3, (4, 5, 64), 5, 2), (7, (3, 4, 6), 4, 4)])
def test_grad_fp32_storage(N, shape, nsteps, ck):
    """FP32 storage: the gradient against the FP64 oracle adjoint (reported;
    the FP32 state rounding bounds it loosely)."""
    say("case adjoint fp32", N, shape, nsteps, ck)
    rng = np.random.default_rng(N * 11 + nsteps)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=((N + 1) ** 2,) + shape)
    tgt = rng.normal(size=shape)
    h, dt = 0.2, 0.07
    L, ga, gs, _ = adj.loss_and_grad(st.Setup(N, shape, h, dt, sa, ss, q), u, nsteps, tgt)
    L2, ga2, gs2 = gpu_grad(N, shape, h, dt, sa, ss, q, u, nsteps, ck, tgt, prec=pm.PM_FP32)
    ea, es = relerr(ga2, ga), relerr(gs2, gs)
    say("  fp32 grad err %.2e %.2e" % (ea, es))
    assert abs(L - L2) <= 1e-5 * L
    assert ea <= 1e-4 and es <= 1e-4


def test_grad_p7_full_vs_c_oracle():
    """The gradient workload at its stated size: P7, 64^3, 200 steps,
    checkpoints every 20 steps; the target is u_0(T) of the oracle run with
    the perturbed sigma_a.  pm_grad against the C oracle adjoint (FP64 to
    1e-11; FP32 storage reported, bound 1e-4), and pm_grad_dev (device
    pointers) equal to pm_grad bit for bit."""
    import workloads
    from gpu_util import progress
    torch = pytest.importorskip("torch")
    w = workloads.p7_adjoint()
    progress("case adjoint p7 %d^3 %d steps, checkpoint %d" % (w.n, w.nsteps, w.checkpoint))
    u0 = w.initial()
    tgt = c_oracle.run(w.N, w.shape, w.h, w.dt, w.extra["perturbed_sigma_a"], w.sigma_s, w.q,
                       u0, w.nsteps)[0]
    progress("adjoint p7: oracle target done")
    L, ga, gs = c_oracle.grad(w.N, w.shape, w.h, w.dt, w.sigma_a, w.sigma_s, w.q, u0, w.nsteps,
                              w.checkpoint, tgt)
    progress("adjoint p7: oracle gradient done")
    dev = torch.device("cuda", 0)
    errs = {}
    for prec in (pm.PM_FP64, pm.PM_FP32):
        gpu_init(w.N, w.shape, w.h, w.dt, w.sigma_a, w.sigma_s, w.q, prec)
        try:
            pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
            for i in range(w.V):
                pm.pm_write(i, u0[i])
            pm.pm_set_checkpoint(w.checkpoint)
            pm.pm_step(w.nsteps)
            u0T = pm.pm_read(0)
            L2 = 0.5 * float(np.sum((u0T - tgt) ** 2))
            ga2, gs2 = pm.pm_grad(u0T - tgt)
            g = torch.from_numpy(u0T - tgt).to(dev)
            da = torch.empty(w.shape, dtype=torch.float64, device=dev)
            ds = torch.empty(w.shape, dtype=torch.float64, device=dev)
            pm.pm_grad_dev(g.data_ptr(), da.data_ptr(), ds.data_ptr())
            assert np.array_equal(da.cpu().numpy(), ga2) and np.array_equal(ds.cpu().numpy(), gs2)
        finally:
            pm.pm_finalize()
            pm.pm_bind_stream(0)
        errs[prec] = (abs(L2 - L) / L, relerr(ga2, ga), relerr(gs2, gs))
        progress("adjoint p7 %s: loss %.2e dsigma_a %.3e dsigma_s %.3e"
                 % ("fp64" if prec == pm.PM_FP64 else "fp32", *errs[prec]))
    assert errs[pm.PM_FP64][0] <= 1e-12
    assert errs[pm.PM_FP64][1] <= 1e-11 and errs[pm.PM_FP64][2] <= 1e-11
    assert errs[pm.PM_FP32][0] <= 1e-5
    assert errs[pm.PM_FP32][1] <= 1e-4 and errs[pm.PM_FP32][2] <= 1e-4
