"""Oracle (test infrastructure only): literal FP64 time stepping in numpy.

Follows Sec. 2.1 of the paper step by step:
  * periodic box of nx x ny x nz equal cells; arrays are indexed [z, y, x]
    (x fastest), matching the flat index x + nx*(y + ny*z);
  * moment i lives on G_{1+o_x, 1+o_y, 1+o_z}; with 0-based cells c its points
    are at (c + 1/2 + o/2) * h, i.e. G111 at cell centres and G211 at
    (c+1) h (the paper's G211 = {i dx} with 1-based i);
  * half-grid centred differences: a target staggered in d (o_d = 1) reads the
    source at c and c+e_d (forward), an unstaggered target reads c-e_d and c
    (backward); indices wrap periodically;
  * eq. (4): every moment of one parity is updated from the frozen differences
    of the dual parity; even parity = even l = G111, G221, G212, G122;
  * eq. (5): exact solution of u' + c u = r over tau,
        u <- u + tau (r - c u) E(-c tau),  E(z) = (exp(z) - 1)/z,  E(0) = 1;
  * eq. (6): one step = S^o_{dt/2} o S^e_{dt} o S^o_{dt/2} (odd half step first).

Medium (Sec. 2, eq. (2) and Sec. 3.2): c = sigma_a for the zeroth moment and
sigma_a + sigma_s for l >= 1 (isotropic scattering); q enters only the zeroth
moment.  Coefficients on staggered points are the arithmetic mean of c over
the 2, 4 or 8 cells that share the point.

Anisotropic scattering (Sec. 2, the slab moment equations): a scattering
kernel that depends only on the angle between the directions acts on degree
l through its Legendre moment Sigma_sl, so the collision coefficient of
degree l is Sigma_a + Sigma_s0 - Sigma_sl.  With Sigma_sl = g_l sigma_s
(g_0 = 1; g_l the moments of a fixed phase function) this is
    c_l = sigma_a + (1 - g_l) sigma_s,
which gives sigma_a for l = 0 and the isotropic case for g_l = 0 (l >= 1).
The same staggered mean is taken of c_l.
"""
import numpy as np

from . import basis

AXIS = {0: -1, 1: -2, 2: -3}   # direction d -> array axis of a [z, y, x] field


def E(z):
    """E(z) = (e^z - 1)/z with E(0) = 1 (eq. (5)); expm1 avoids cancellation."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


class Setup:
    """Everything the literal step needs, derived from the paper's definitions."""

    def __init__(self, N, shape, h, dt, sigma_a, sigma_s, q=None, scattering=None):
        """scattering: g_l for l = 1, 2, ... (None: isotropic; degrees past
        the sequence and past N are isotropic / unused)."""
        self.N = N
        self.V = basis.n_moments(N)
        self.shape = tuple(shape)            # (nz, ny, nx)
        self.h = (float(h),) * 3 if np.isscalar(h) else tuple(float(v) for v in h)  # (hx, hy, hz)
        self.dt = float(dt)
        self.M = basis.flux_matrices(N)
        self.o = basis.reflection_parities(N)
        self.ell = np.array([basis.lm_of(i)[0] for i in range(self.V)])
        self.parity = self.o.sum(axis=1) % 2          # 0 = even grids, 1 = odd grids
        sa = np.asarray(sigma_a, dtype=np.float64).reshape(self.shape)
        ss = np.asarray(sigma_s, dtype=np.float64).reshape(self.shape)
        self.sigma_a, self.sigma_s = sa, ss
        self.q = (np.zeros(self.shape) if q is None
                  else np.asarray(q, dtype=np.float64).reshape(self.shape))
        self.g = scattering_moments(N, scattering)
        self.cbar = []
        for i in range(self.V):
            c = sa if i == 0 else sa + (1.0 - self.g[self.ell[i]]) * ss
            self.cbar.append(staggered_mean(c, self.o[i]))
        self.targets = {p: [i for i in range(self.V) if self.parity[i] == p] for p in (0, 1)}
        self.sources = {}
        for i in range(self.V):
            self.sources[i] = [(d, j, self.M[d][i, j]) for d in range(3)
                               for j in np.nonzero(self.M[d][i])[0]]


def scattering_moments(N, scattering):
    """g_0 .. g_N: g_0 = 1, then the given g_l for l >= 1, zero past them."""
    g = np.zeros(N + 1)
    g[0] = 1.0
    if scattering is not None:
        vals = np.asarray(scattering, dtype=np.float64).ravel()
        k = min(N, vals.size)
        g[1:k + 1] = vals[:k]
    return g


def staggered_mean(c, o):
    """Mean of a cell-centred field over the cells sharing a staggered point."""
    acc = c.copy()
    n = 1
    for d in range(3):
        if o[d]:
            acc = acc + np.roll(acc, -1, axis=AXIS[d])
            n *= 2
    return acc / n


def difference(u, d, target_staggered, h):
    """Half-grid centred difference in direction d, landing on the target grid."""
    ax = AXIS[d]
    if target_staggered:
        return (np.roll(u, -1, axis=ax) - u) / h
    return (u - np.roll(u, 1, axis=ax)) / h


def residual(s, u, i):
    """r_i = q_i - sum_d sum_j M_d[i, j] D_d u_j  (right-hand side of eq. (4))."""
    r = s.q.copy() if i == 0 else np.zeros(s.shape)
    for d, j, mij in s.sources[i]:
        r -= mij * difference(u[j], d, s.o[i][d] == 1, s.h[d])
    return r


def substep(s, u, parity, tau):
    """S^parity_tau: eq. (5) applied to every moment of the given parity."""
    r = {i: residual(s, u, i) for i in s.targets[parity]}
    for i, ri in r.items():
        c = s.cbar[i]
        u[i] = u[i] + tau * (ri - c * u[i]) * E(-c * tau)
    return u


def step(s, u):
    """One Strang step, eq. (6): odd half step, even full step, odd half step."""
    substep(s, u, 1, 0.5 * s.dt)
    substep(s, u, 0, s.dt)
    substep(s, u, 1, 0.5 * s.dt)
    return u


def run(s, u0, nsteps):
    u = np.array(u0, dtype=np.float64, copy=True).reshape((s.V,) + s.shape)
    for _ in range(nsteps):
        step(s, u)
    return u
