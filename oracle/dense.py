"""Oracle (test infrastructure only): explicit step matrices on tiny grids.

An independent assembly of the same scheme (Sec. 2.1, eq. (4)-(6)): instead
of shifting arrays, the one-dimensional periodic difference operators are
built as matrices and combined by Kronecker products; a substep becomes an
affine map u -> A u + b with
    A_ii = diag(alpha_i),  A_ij = -diag(beta_i) M_d[i, j] D_d   (i target, j dual),
    alpha = exp(-c tau),   beta = tau E(-c tau),
which is eq. (5) rewritten (1 - c tau E(-c tau) = exp(-c tau)).

Also the Fourier symbol of the step for a homogeneous medium: a plane wave
with wave vector k is an eigenfunction of every difference operator; on the
staggered points the symbol of a half-grid difference is 2 i sin(k_d h_d/2)/h_d.
"""
import numpy as np
import scipy.sparse as sp

from . import basis
from .stepper import E


def diff_1d(n, h, forward):
    """Periodic half-grid difference on n points as a sparse n x n matrix."""
    I = sp.identity(n, format="csr")
    if forward:      # (u[c+1] - u[c]) / h
        S = sp.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) + 1) % n)), shape=(n, n))
        return (S - I) / h
    S = sp.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) - 1) % n)), shape=(n, n))
    return (I - S) / h


def diff_3d(shape, h, d, forward):
    nz, ny, nx = shape
    Iz, Iy, Ix = (sp.identity(k, format="csr") for k in (nz, ny, nx))
    if d == 0:
        return sp.kron(Iz, sp.kron(Iy, diff_1d(nx, h[0], forward)))
    if d == 1:
        return sp.kron(Iz, sp.kron(diff_1d(ny, h[1], forward), Ix))
    return sp.kron(diff_1d(nz, h[2], forward), sp.kron(Iy, Ix))


def substep_matrix(s, parity, tau):
    """(A, b) of one substep S^parity_tau as a sparse matrix over [moment, cell]."""
    V = s.V
    ncell = int(np.prod(s.shape))
    blocks = [[None] * V for _ in range(V)]
    b = np.zeros(V * ncell)
    D = {(d, f): diff_3d(s.shape, s.h, d, f) for d in range(3) for f in (False, True)}
    for i in range(V):
        if s.parity[i] != parity:
            blocks[i][i] = sp.identity(ncell, format="csr")
            continue
        c = s.cbar[i].ravel()
        alpha = np.exp(-c * tau)
        beta = tau * E(-c * tau)
        blocks[i][i] = sp.diags(alpha)
        Bi = sp.diags(beta)
        for d in range(3):
            for j in np.nonzero(s.M[d][i])[0]:
                term = -s.M[d][i, j] * (Bi @ D[(d, bool(s.o[i][d]))])
                blocks[i][j] = term if blocks[i][j] is None else blocks[i][j] + term
        if i == 0:
            b[:ncell] = beta * s.q.ravel()
    return sp.bmat(blocks, format="csr"), b


def step_matrix(s):
    """Affine map of one Strang step (eq. (6)) as (S, b): u_new = S u + b."""
    Ao, bo = substep_matrix(s, 1, 0.5 * s.dt)
    Ae, be = substep_matrix(s, 0, s.dt)
    S = Ao @ Ae @ Ao
    b = Ao @ (Ae @ bo + be) + bo
    return S, b


def fourier_symbol(N, k, h, dt, c0, c1, c_deg=None):
    """V x V amplification matrix of one step for a homogeneous medium.

    k: wave vector (kx, ky, kz); h: (hx, hy, hz); c0 = coefficient of the
    zeroth moment, c1 = coefficient of all l >= 1 moments; c_deg, when
    given, replaces both with one coefficient per degree l = 0..N
    (anisotropic scattering); no source.  Amplitudes are referred to each
    moment's own staggered points.
    """
    Mx, My, Mz = basis.flux_matrices(N)
    o = basis.reflection_parities(N)
    parity = o.sum(axis=1) % 2
    V = basis.n_moments(N)
    kappa = [2.0j * np.sin(0.5 * k[d] * h[d]) / h[d] for d in range(3)]
    L = kappa[0] * Mx + kappa[1] * My + kappa[2] * Mz
    c = np.full(V, float(c1))
    c[0] = c0
    if c_deg is not None:
        c = np.array([float(c_deg[basis.lm_of(i)[0]]) for i in range(V)])

    def sub(p, tau):
        A = np.eye(V, dtype=complex)
        for i in range(V):
            if parity[i] != p:
                continue
            alpha = np.exp(-c[i] * tau)
            beta = tau * E(-c[i] * tau)
            A[i, :] = -beta * L[i, :]
            A[i, i] = alpha
        return A

    Ao = sub(1, 0.5 * dt)
    Ae = sub(0, dt)
    return Ao @ Ae @ Ao


def staggered_positions(shape, h, o):
    """Coordinates (x, y, z) of the points of a moment with parities o."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x + 0.5 + 0.5 * o[0]) * h[0], (y + 0.5 + 0.5 * o[1]) * h[1],
            (z + 0.5 + 0.5 * o[2]) * h[2])
