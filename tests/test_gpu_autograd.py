"""Differentiation form: the torch.autograd.Function over the C ABI against
the oracle adjoint and against central finite differences of the GPU
forward (the gradient workload: P7, 64^3, 200 steps, checkpoints every 20)."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm
import workloads
from oracle import adjoint as adj
from oracle import stepper as st

from gpu_util import gpu_run, relerr, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def loss_grad_autograd(sa, ss, q, u0, N, h, dt, nsteps, ck, target, prec=0):
    from paper_2004_02833_amd.autograd import run_u0
    dev = torch.device("cuda", 0)
    tsa = torch.tensor(sa, device=dev, requires_grad=True)
    tss = torch.tensor(ss, device=dev, requires_grad=True)
    spec = dict(N=N, dx=h, dt=dt, nsteps=nsteps, checkpoint=ck, q=q, precision=prec,
                moments=(lambda i: u0(i)) if callable(u0) else (lambda i: u0[i]))
    u0T = run_u0(tsa, tss, spec)
    tg = torch.tensor(target, device=dev)
    L = 0.5 * ((u0T - tg) ** 2).sum()
    L.backward()
    out = (float(L.detach()), tsa.grad.cpu().numpy(), tss.grad.cpu().numpy())
    pm.pm_finalize()
    return out


def test_autograd_matches_oracle_adjoint():
    N, shape = 3, (4, 5, 6)
    rng = np.random.default_rng(70)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=(16,) + shape)
    tgt = rng.normal(size=shape)
    h, dt = 0.2, 0.07
    L, ga, gs, _ = adj.loss_and_grad(st.Setup(N, shape, h, dt, sa, ss, q), u, 6, tgt)
    L2, ga2, gs2 = loss_grad_autograd(sa, ss, q, u, N, h, dt, 6, 4, tgt)
    assert abs(L - L2) <= 1e-13 * L
    assert relerr(ga2, ga) <= 1e-12 and relerr(gs2, gs) <= 1e-12


def fd_gradients(w, target, cells, which, hs, prec=0):
    """Central differences (L+ - L-)/(2h) written as
    sum (u+ - u-) (0.5 (u+ + u-) - target) / (2h), which is exact algebra and
    avoids the cancellation of two large losses."""
    out = {}
    for cell in cells:
        vals = []
        for h in hs:
            res = []
            for sgn in (1, -1):
                sa = w.sigma_a.copy()
                ss = w.sigma_s.copy()
                (sa if which == "a" else ss)[cell] += sgn * h
                res.append(gpu_run(w.N, w.shape, w.h, w.dt, sa, ss, w.q, w.moment, w.nsteps,
                                   prec=prec, moments=[0])[0])
            up, um = res
            vals.append(float(np.sum((up - um) * (0.5 * (up + um) - target)) / (2 * h)))
        out[cell] = vals
    return out


@pytest.mark.parametrize("n,nsteps,ncell", [(64, 200, 16)])
def test_gradient_workload_vs_finite_differences(n, nsteps, ncell):
    """P7 gradient workload: autograd dL/dsigma_a, dL/dsigma_s against central
    differences on seeded cells; the FD value closest to the adjoint over the
    step sizes (the plateau) must agree to 1e-6 relative."""
    w = workloads.p7_adjoint(n=n, nsteps=nsteps)
    say("case gradient workload %d^3 %d steps" % (n, nsteps))
    target = gpu_run(w.N, w.shape, w.h, w.dt, w.extra["perturbed_sigma_a"], w.sigma_s, w.q,
                     w.moment, w.nsteps, moments=[0])[0]
    L, ga, gs = loss_grad_autograd(w.sigma_a, w.sigma_s, w.q, w.moment, w.N, w.h, w.dt,
                                   w.nsteps, w.checkpoint, target)
    rng = np.random.default_rng(123)
    cells = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(ncell)]
    hs = (1e-3, 3e-4, 1e-4, 3e-5)
    worst = 0.0
    for which, G in (("a", ga), ("s", gs)):
        fd = fd_gradients(w, target, cells, which, hs)
        for cell, vals in fd.items():
            g = G[cell]
            best = min(abs(v - g) for v in vals)
            scale = max(abs(g), 1e-3 * np.abs(G).max())
            worst = max(worst, best / scale)
            say("  d/dsigma_%s %s adjoint %.10e fd %s" % (which, cell, g, ["%.10e" % v for v in vals]))
    say("worst FD rel err", worst)
    assert worst <= 1e-6


def test_backward_after_another_forward_raises():
    """The library keeps one recording: a backward whose forward has been
    replaced by another forward raises instead of returning the other run's
    gradients; the later forward's backward still works."""
    from paper_2004_02833_amd.autograd import StaleRecordingError, run_u0
    N, shape = 3, (4, 5, 64)
    rng = np.random.default_rng(71)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=(16,) + shape)
    dev = torch.device("cuda", 0)
    spec = dict(N=N, dx=0.2, dt=0.07, nsteps=5, checkpoint=2, q=q, moments=lambda i: u[i])
    sa1 = torch.tensor(rng.uniform(0, 0.5, shape), device=dev, requires_grad=True)
    ss1 = torch.tensor(rng.uniform(0, 1, shape), device=dev, requires_grad=True)
    sa2 = torch.tensor(rng.uniform(0, 0.5, shape), device=dev, requires_grad=True)
    ss2 = torch.tensor(rng.uniform(0, 1, shape), device=dev, requires_grad=True)
    try:
        y1 = run_u0(sa1, ss1, spec)
        y2 = run_u0(sa2, ss2, spec)
        with pytest.raises(StaleRecordingError):
            y1.sum().backward()
        y2.sum().backward()
        assert sa2.grad is not None and torch.isfinite(sa2.grad).all()
        # extending the recording also invalidates it
        y3 = run_u0(sa1, ss1, spec)
        pm.pm_step(1)
        with pytest.raises(StaleRecordingError):
            y3.sum().backward()
    finally:
        pm.pm_finalize()
