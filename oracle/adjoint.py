"""Oracle (test infrastructure only): adjoint of the literal step and gradients.

The paper does not treat derivatives; this follows from its scheme by the
chain rule.  For one substep S^F_tau (eq. (4)-(5)) with target moments i of
parity F,
    u_i' = alpha_i u_i + beta_i r_i,   r_i = q_i - sum_d sum_j M_d[i,j] D_d u_j,
the transposed map applied to a cotangent lam (of u') is
    g_alpha_i += lam_i * u_i          g_beta_i += lam_i * r_i
    lam_j     += - sum_i sum_d M_d[i,j] D_d^T (beta_i lam_i)     (j dual)
    lam_i      = alpha_i lam_i
with D_d^T the matrix transpose of the periodic one-sided difference.  The
coefficients depend on the medium through c = mean of
sigma_a + (1 - g_l) sigma_s over the cells sharing a point (g_0 = 1; g_l = 0
for l >= 1 with isotropic scattering):
    d alpha/dc = -tau alpha,   d beta/dc = (tau alpha - beta)/c  (-> -tau^2/2).
Loss: L = 1/2 sum_cells (u_0(T) - target)^2, no cell-volume weight.
"""
import numpy as np

from . import stepper
from .stepper import AXIS, E


def difference_T(v, d, target_staggered, h):
    """Transpose of stepper.difference (periodic)."""
    ax = AXIS[d]
    if target_staggered:     # D v = (v[c+1] - v[c])/h  ->  D^T w = (w[c-1] - w[c])/h
        return (np.roll(v, 1, axis=ax) - v) / h
    return (v - np.roll(v, -1, axis=ax)) / h   # D v = (v[c]-v[c-1])/h -> (w[c]-w[c+1])/h


def dbeta_dc(c, tau):
    """Derivative of beta = tau E(-c tau) with respect to c."""
    c = np.asarray(c, dtype=np.float64)
    z = c * tau
    out = np.empty_like(c)
    small = np.abs(z) < 1e-3
    zs = z[small]
    out[small] = tau * tau * (-0.5 + zs / 3.0 - zs * zs / 8.0 + zs ** 3 / 30.0)
    cl = c[~small]
    alpha = np.exp(-cl * tau)
    beta = -np.expm1(-cl * tau) / cl
    out[~small] = (tau * alpha - beta) / cl
    return out


def staggered_mean_T(g, o):
    """Transpose of stepper.staggered_mean."""
    acc = g.copy()
    n = 1
    for d in range(3):
        if o[d]:
            acc = acc + np.roll(acc, 1, axis=AXIS[d])
            n *= 2
    return acc / n


def substep_T(s, u_old, lam, parity, tau, gc):
    """Transpose of one substep; accumulates dL/dc per moment into gc[i]."""
    tg = s.targets[parity]
    for i in tg:
        c = s.cbar[i]
        alpha = np.exp(-c * tau)
        beta = tau * E(-c * tau)
        r = stepper.residual(s, u_old, i)
        ga = lam[i] * u_old[i]
        gb = lam[i] * r
        gc[i] += ga * (-tau * alpha) + gb * dbeta_dc(c, tau)
        w = beta * lam[i]
        for d, j, mij in s.sources[i]:
            lam[j] -= mij * difference_T(w, d, s.o[i][d] == 1, s.h[d])
    for i in tg:
        c = s.cbar[i]
        lam[i] = np.exp(-c * tau) * lam[i]
    return lam


def loss_and_grad(s, u0, nsteps, target):
    """L and (dL/dsigma_a, dL/dsigma_s) for L = 1/2 ||u_0(T) - target||^2."""
    u = np.array(u0, dtype=np.float64, copy=True).reshape((s.V,) + s.shape)
    tape = []
    seq = [(1, 0.5 * s.dt), (0, s.dt), (1, 0.5 * s.dt)]
    for _ in range(nsteps):
        for p, tau in seq:
            tape.append((u.copy(), p, tau))
            stepper.substep(s, u, p, tau)
    diff = u[0] - np.asarray(target).reshape(s.shape)
    L = 0.5 * float(np.sum(diff * diff))
    lam = np.zeros_like(u)
    lam[0] = diff
    gc = np.zeros_like(u)
    for u_old, p, tau in reversed(tape):
        substep_T(s, u_old, lam, p, tau, gc)
    ga = np.zeros(s.shape)
    gs = np.zeros(s.shape)
    for i in range(s.V):
        g = staggered_mean_T(gc[i], s.o[i])
        ga += g
        gs += (1.0 - s.g[s.ell[i]]) * g
    return L, ga, gs, lam
