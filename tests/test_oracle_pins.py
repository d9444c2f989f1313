"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here touches the HIP path.  Each test names the passage or the fact
it checks; together they are chosen so that a dropped term, a wrong sign,
index or orientation, or a transposed operand in the oracle fails one of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import basis, dense
from oracle import stepper as st

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


# ---------------------------------------------------------------- basis ----

def test_separable_harmonics_match_scipy():
    """Long-double R_i (own recurrences) == scipy's Y_l^m combination, l <= 39."""
    rng = np.random.default_rng(0)
    mu = rng.uniform(-1, 1, 40)
    ph = rng.uniform(0, 2 * np.pi, 40)
    A = basis.real_sh(39, mu, ph)
    B = basis.separable_sh(39, mu, ph).astype(np.float64)
    assert np.abs(A - B).max() < 1e-11 * np.abs(A).max()


def test_low_order_harmonics_closed_form():
    """R_00 = 1/sqrt(4 pi); R_{1,1}, R_{1,-1}, R_{1,0} = sqrt(3/(4 pi)) (Om_x, Om_y, Om_z)."""
    rng = np.random.default_rng(1)
    mu = rng.uniform(-1, 1, 10)
    ph = rng.uniform(0, 2 * np.pi, 10)
    ox, oy, oz = basis.directions(mu, ph)
    R = basis.real_sh(1, mu, ph)
    c = np.sqrt(3 / (4 * np.pi))
    assert np.allclose(R[0], 1 / np.sqrt(4 * np.pi), atol=1e-15)
    assert np.allclose(R[basis.moment_index(1, 1)], c * ox, atol=1e-15)
    assert np.allclose(R[basis.moment_index(1, -1)], c * oy, atol=1e-15)
    assert np.allclose(R[basis.moment_index(1, 0)], c * oz, atol=1e-15)


@pytest.mark.parametrize("N", [3, 7])
def test_basis_orthonormal(N):
    assert np.abs(basis.gram_matrix(N) - np.eye(basis.n_moments(N))).max() < 1e-13


def test_gauss_legendre_long_double():
    x, w = basis.gauss_legendre_ld(12)
    xd, wd = np.polynomial.legendre.leggauss(12)
    assert np.abs(x.astype(float) - xd).max() < 1e-15
    # exact for x^22: integral = 2/23
    assert abs(float(np.sum(w * x ** 22)) - 2 / 23) < 1e-17


@pytest.fixture(scope="module")
def mats():
    return {N: basis.flux_matrices(N) for N in (1, 2, 3, 7, 39)}


@pytest.mark.parametrize("N", [1, 3, 7, 39])
def test_flux_symmetric(mats, N):
    """Eq. (3): the system matrices are symmetric."""
    for M in mats[N]:
        assert np.array_equal(M, M.T) or np.abs(M - M.T).max() < 1e-16


def test_flux_spot_values(mats):
    """M_x[(0,0),(1,1)] = M_y[(0,0),(1,-1)] = M_z[(0,0),(1,0)] = 1/sqrt(3)."""
    Mx, My, Mz = mats[3]
    i = basis.moment_index
    for M, j in ((Mx, i(1, 1)), (My, i(1, -1)), (Mz, i(1, 0))):
        assert abs(M[0, j] - 1 / np.sqrt(3)) <= 2.3e-16
        assert np.count_nonzero(M[0]) == 1


@pytest.mark.parametrize("N", [3, 7, 39])
def test_nnz_per_row_as_printed(mats, N):
    """Sec. 3.2: M_x, M_y have 1..4 nonzeros per row, M_z 0..2, total <= 10."""
    g = GOLD["nnz_per_row"]["value"]
    Mx, My, Mz = mats[N]
    cx = np.count_nonzero(Mx, axis=1)
    cy = np.count_nonzero(My, axis=1)
    cz = np.count_nonzero(Mz, axis=1)
    assert cx.min() >= g["Mx"][0] and cx.max() <= g["Mx"][1]
    assert cy.min() >= g["My"][0] and cy.max() <= g["My"][1]
    assert cz.min() >= g["Mz"][0] and cz.max() <= g["Mz"][1]
    assert (cx + cy + cz).max() <= g["max_total"]
    total = {3: 70, 7: 438, 39: 14902}[N]
    assert int(cx.sum() + cy.sum() + cz.sum()) == total


def test_moment_count_P39():
    assert basis.n_moments(39) == GOLD["moments_P39"]["value"]


def legendre_1d(N):
    """Tridiagonal M of the slab recursion in Sec. 2 (Legendre moments)."""
    L = np.zeros((N + 1, N + 1))
    for l in range(N + 1):
        if l + 1 <= N:
            L[l, l + 1] = (l + 1) / (2 * l + 1)
        if l - 1 >= 0:
            L[l, l - 1] = l / (2 * l + 1)
    return L


@pytest.mark.parametrize("N", [1, 3, 7, 39])
def test_1d_legendre_spectrum_and_mz_block(mats, N):
    """Eigenvalues of the slab P_N matrix are the N+1 Gauss-Legendre nodes, and
    the m = 0 block of M_z is that matrix in orthonormal scaling."""
    nodes = np.polynomial.legendre.leggauss(N + 1)[0]
    ev = np.sort(np.linalg.eigvals(legendre_1d(N)).real)
    assert np.abs(ev - nodes).max() < 1e-12
    Mz = mats[N][2]
    idx = [basis.moment_index(l, 0) for l in range(N + 1)]
    B = Mz[np.ix_(idx, idx)]
    # u_l = 2 pi sqrt((2l+1)/(4 pi)) psi_l  =>  B = S L S^-1
    S = np.diag([np.sqrt((2 * l + 1) / (4 * np.pi)) for l in range(N + 1)])
    assert np.abs(B - S @ legendre_1d(N) @ np.linalg.inv(S)).max() < 1e-14


@pytest.mark.parametrize("N", [3, 7])
def test_rotational_invariance(mats, N):
    """spec(n . M) = spec(M_z) for any unit n (rotational invariance of P_N)."""
    Mx, My, Mz = mats[N]
    ref = np.sort(np.linalg.eigvalsh(Mz))
    rng = np.random.default_rng(N)
    for _ in range(3):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        ev = np.sort(np.linalg.eigvalsh(n[0] * Mx + n[1] * My + n[2] * Mz))
        assert np.abs(ev - ref).max() < 1e-13
    lam = {3: 0.861136, 7: 0.960290}[N]
    assert abs(ref.max() - np.polynomial.legendre.leggauss(N + 1)[0].max()) < 1e-13
    assert abs(ref.max() - lam) < 1e-6


@pytest.mark.parametrize("N", [3, 7])
def test_closure_on_interior_rows(mats, N):
    """Om_x^2 + Om_y^2 + Om_z^2 = 1: sum_d M_d^2 = I on rows with l < N."""
    S = sum(M @ M for M in mats[N])
    for i in range(basis.n_moments(N)):
        if basis.lm_of(i)[0] < N:
            e = np.zeros(basis.n_moments(N))
            e[i] = 1
            assert np.abs(S[i] - e).max() < 1e-14


@pytest.mark.parametrize("N", [2, 3, 7, 39])
def test_families_follow_coupling(mats, N):
    """Sec. 2.1: a d-derivative couples grids that differ in exactly index d;
    u_0 lives on G111; even grids hold the even-l moments."""
    o = basis.reflection_parities(N)
    for d, M in enumerate(mats[N]):
        ii, jj = np.nonzero(M)
        diff = o[ii] ^ o[jj]
        expect = np.zeros(3, dtype=int)
        expect[d] = 1
        assert np.all(diff == expect)
    assert basis.family_name(o[0]) == GOLD["zeroth_moment_grid"]["value"]
    fam = basis.families(N)
    even = set(GOLD["even_grids"]["value"])
    odd = set(GOLD["odd_grids"]["value"])
    for i, f in enumerate(fam):
        l = basis.lm_of(i)[0]
        assert f in (even if l % 2 == 0 else odd)


def test_family_sizes():
    sizes = {3: [3, 1, 1, 1, 3, 3, 3, 1], 7: [10, 6, 6, 6, 10, 10, 10, 6],
             39: [210, 190, 190, 190, 210, 210, 210, 190]}
    for N, want in sizes.items():
        fam = basis.families(N)
        got = [fam.count(g) for g in GOLD["storage_order"]["value"]]
        assert got == want


def test_flop_model_counts():
    """Sec. 5.1.1 prints 68.3/50.5/45.1 FLOP per LCUP for 392 + 40 a + 50 b
    FLOP per cell-step; with a = #odd-l and b = #even-l moments of the basis
    the printed averages are reproduced (labels in the text are swapped)."""
    g = GOLD["flop_model"]["value"]
    for N, want in g["flop_per_lcup"].items():
        N = int(N)
        fam = basis.families(N)
        n_even = sum(f in GOLD["even_grids"]["value"] for f in fam)
        n_odd = len(fam) - n_even
        val = (g["base"] + g["per_a"] * n_odd + g["per_b"] * n_even) / len(fam)
        assert abs(val - want) < 0.05


# ---------------------------------------------------------------- step -----

def test_E_function():
    """eq. (5): E(0) = 1 exactly; E continuous at 0; E(z) = (e^z - 1)/z."""
    assert st.E(np.array([0.0]))[0] == 1.0
    z = np.array([1e-300, -1e-12, 1e-8, -0.5, 3.0])
    ref = np.array([1.0, 1 - 0.5e-12, 1 + 0.5e-8, (np.exp(-0.5) - 1) / -0.5, (np.exp(3) - 1) / 3])
    assert np.allclose(st.E(z), ref, rtol=1e-15, atol=0)


def _setup(N, shape, seed, h=0.25, dt=0.08, q=False, sa_zero=False):
    rng = np.random.default_rng(seed)
    sa = np.zeros(shape) if sa_zero else rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    qq = rng.uniform(0, 1, shape) if q else None
    s = st.Setup(N, shape, h, dt, sa, ss, qq)
    u = rng.normal(size=(s.V,) + tuple(shape))
    return s, u


@pytest.mark.parametrize("N,shape", [(1, (4, 4, 4)), (3, (4, 4, 4)), (3, (2, 3, 4)), (2, (1, 1, 5)),
                                     (3, (3, 1, 1)), (2, (1, 4, 1))])
def test_dense_matrix_equals_stepping(N, shape):
    """Independent Kronecker-product assembly of eq. (4)-(6) == array stepping."""
    s, u = _setup(N, shape, 7, q=True)
    S, b = dense.step_matrix(s)
    x = u.ravel().copy()
    for _ in range(3):
        x = S @ x + b
    y = st.run(s, u, 3).ravel()
    assert np.abs(x - y).max() <= 1e-13 * np.abs(x).max()


def test_dense_step_contractive_below_cfl():
    """|lambda(S)| <= 1 for sigma >= 0 and dt below the stability limit."""
    s, _ = _setup(3, (4, 4, 4), 8, h=0.25, dt=0.5 * 0.25)
    S, _ = dense.step_matrix(s)
    ev = np.linalg.eigvals(S.toarray())
    assert np.abs(ev).max() <= 1 + 1e-12


def test_conservation_zero_absorption():
    """sigma_a = 0, q = 0: sum of u_0 over the periodic box is constant."""
    s, u = _setup(3, (4, 5, 6), 9, sa_zero=True)
    tot = u[0].sum()
    v = u.copy()
    for _ in range(20):
        st.step(s, v)
        assert abs(v[0].sum() - tot) < 1e-14 * np.abs(u[0]).sum()


def test_conservation_with_source():
    """sigma_a = 0: the even full step adds exactly dt * sum(q) to sum(u_0)."""
    s, u = _setup(3, (4, 5, 6), 10, sa_zero=True, q=True)
    v = u.copy()
    for k in range(1, 6):
        st.step(s, v)
        want = u[0].sum() + k * s.dt * s.q.sum()
        assert abs(v[0].sum() - want) < 1e-13 * abs(want)


def test_homogeneous_decay_exact():
    """Homogeneous state and medium: u_0 ~ exp(-sigma_a t), u_{l>=1} ~ exp(-(sigma_a + sigma_s) t);
    with a source u_0 = q/sa + (u_0(0) - q/sa) exp(-sa t)."""
    N, shape = 3, (3, 3, 3)
    sa, ss, qv = 0.7, 1.3, 0.4
    s = st.Setup(N, shape, 0.2, 0.05, np.full(shape, sa), np.full(shape, ss), np.full(shape, qv))
    u0 = np.arange(1.0, 17.0)[:, None, None, None] * np.ones((16,) + shape)
    v = u0.copy()
    for k in range(1, 11):
        st.step(s, v)
        t = k * s.dt
        want0 = qv / sa + (1.0 - qv / sa) * np.exp(-sa * t)
        assert np.abs(v[0] - want0).max() < 1e-14
        want = u0[1:, 0, 0, 0] * np.exp(-(sa + ss) * t)
        assert np.abs(v[1:, 0, 0, 0] - want).max() < 1e-14 * 16


@pytest.mark.parametrize("N,kv", [(3, (1, 2, 3)), (3, (2, -1, 1)), (2, (0, 0, 1)), (3, (3, 0, -2))])
def test_fourier_mode(N, kv):
    """A plane wave on a homogeneous medium evolves by the Strang product of
    the substep symbols (difference symbol 2 i sin(k h/2)/h)."""
    shape = (6, 6, 6)
    h = 1.0 / 6
    dt = 0.4 * h
    c0, c1 = 0.3, 0.9
    sa = np.full(shape, c0)
    ss = np.full(shape, c1 - c0)
    s = st.Setup(N, shape, h, dt, sa, ss)
    k = 2 * np.pi * np.array(kv, dtype=float)
    rng = np.random.default_rng(11)
    uh = rng.normal(size=s.V) + 1j * rng.normal(size=s.V)
    ph = np.empty((s.V,) + shape, dtype=complex)
    for i in range(s.V):
        x, y, z = dense.staggered_positions(shape, (h, h, h), s.o[i])
        ph[i] = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    u = (uh[:, None, None, None] * ph).real
    nsteps = 5
    G = dense.fourier_symbol(N, k, (h, h, h), dt, c0, c1)
    want = ((np.linalg.matrix_power(G, nsteps) @ uh)[:, None, None, None] * ph).real
    got = st.run(s, u, nsteps)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("N", [1, 3, 7])
def test_cfl_limit_from_symbol(N):
    """sigma = 0: the step is stable (spectral radius 1) iff
    dt <= h / (sqrt(3) lambda_max(N)); the paper's dt < h/3 is sufficient."""
    h = 1.0
    lam = np.polynomial.legendre.leggauss(N + 1)[0].max()
    lim = h / (np.sqrt(3) * lam)
    assert lim > GOLD["cfl_sufficient"]["value"] * h
    ks = np.linspace(0, np.pi, 5)
    def radius(dt):
        r = 0.0
        for kx in ks:
            for ky in ks:
                for kz in ks:
                    G = dense.fourier_symbol(N, (kx, ky, kz), (h, h, h), dt, 0.0, 0.0)
                    r = max(r, np.abs(np.linalg.eigvals(G)).max())
        return r
    assert radius(0.98 * lim) <= 1 + 1e-10
    assert radius(1.05 * lim) > 1 + 1e-6


def slab_pn(N, n, h, dt, psi0, steps, sa, ss):
    """Independent 1D staggered P_N in Legendre moments psi_l (Sec. 2, eq. (2)),
    written with loops: even l at cell centres, odd l at faces (c+1) h."""
    L = legendre_1d(N)
    psi = [list(p) for p in psi0]
    c = [sa] + [sa + ss] * N
    def sub(par, tau):
        new = [row[:] for row in psi]
        for l in range(N + 1):
            if l % 2 != par:
                continue
            cl = c[l]
            Ef = 1.0 if cl == 0 else np.expm1(-cl * tau) / (-cl * tau)
            for x in range(n):
                r = 0.0
                for j in (l - 1, l + 1):
                    if 0 <= j <= N:
                        if par == 1:   # target on faces: forward
                            dd = (psi[j][(x + 1) % n] - psi[j][x]) / h
                        else:
                            dd = (psi[j][x] - psi[j][(x - 1) % n]) / h
                        r -= L[l, j] * dd
                new[l][x] = psi[l][x] + tau * (r - cl * psi[l][x]) * Ef
        psi[:] = new
    for _ in range(steps):
        sub(1, 0.5 * dt)
        sub(0, dt)
        sub(1, 0.5 * dt)
    return np.array(psi)


def test_1d_reduction_matches_slab_pn():
    """nx = ny = 1: only M_z acts and the m = 0 moments follow the slab P_N of
    Sec. 2 (eq. (2) with the three-term recursion), up to the scaling
    u_l = 2 pi sqrt((2l+1)/(4 pi)) psi_l."""
    N, n = 5, 12
    h, dt = 1.0 / n, 0.4 / n
    sa, ss = 0.3, 0.8
    shape = (n, 1, 1)
    s = st.Setup(N, shape, h, dt, np.full(shape, sa), np.full(shape, ss))
    rng = np.random.default_rng(12)
    psi0 = rng.normal(size=(N + 1, n))
    u = np.zeros((s.V,) + shape)
    scale = [2 * np.pi * np.sqrt((2 * l + 1) / (4 * np.pi)) for l in range(N + 1)]
    for l in range(N + 1):
        u[basis.moment_index(l, 0), :, 0, 0] = scale[l] * psi0[l]
    got = st.run(s, u, 7)
    want = slab_pn(N, n, h, dt, psi0, 7, sa, ss)
    for l in range(N + 1):
        assert np.abs(got[basis.moment_index(l, 0), :, 0, 0] - scale[l] * want[l]).max() < 1e-13
    # the m != 0 moments stay zero
    mask = np.ones(s.V, bool)
    mask[[basis.moment_index(l, 0) for l in range(N + 1)]] = False
    assert np.abs(got[mask]).max() == 0.0


def mirror(u, o, d, cell_centred=False):
    """Reflection x_d -> -x_d of a staggered field (periodic box)."""
    ax = st.AXIS[d]
    n = u.shape[ax]
    if cell_centred or not o:
        idx = (n - 1 - np.arange(n)) % n
    else:
        idx = (n - 2 - np.arange(n)) % n
    return np.take(u, idx, axis=ax)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_mirror_symmetry(d):
    """Reflecting space and Omega_d together commutes with the step: moments
    odd under the reflection change sign, staggered points map c -> n-2-c."""
    N, shape = 3, (4, 5, 6)
    rng = np.random.default_rng(20 + d)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    s = st.Setup(N, shape, 0.2, 0.06, sa, ss, q)
    u = rng.normal(size=(s.V,) + shape)
    def M(v):
        return np.stack([(-1) ** s.o[i][d] * mirror(v[i], s.o[i][d], d) for i in range(s.V)])
    sm = st.Setup(N, shape, 0.2, 0.06, mirror(sa, 0, d, True), mirror(ss, 0, d, True),
                  mirror(q, 0, d, True))
    a = M(st.run(s, u, 3))
    b = st.run(sm, M(u), 3)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_swap_xy_symmetry():
    """Exchanging x and y (Omega_x <-> Omega_y) maps the moments by the
    orthogonal matrix T_ij = int R_i(Om) R_j(swap Om) and commutes with the step."""
    N, shape = 3, (3, 4, 4)
    mu, ph, w = basis.sphere_rule(N)
    R = basis.real_sh(N, mu, ph)
    Rs = basis.real_sh(N, mu, np.pi / 2 - ph)
    T = (R * w) @ Rs.T
    T[np.abs(T) < 1e-12] = 0
    assert np.abs(T @ T.T - np.eye(16)).max() < 1e-12
    rng = np.random.default_rng(30)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    s = st.Setup(N, shape, 0.2, 0.06, sa, ss)
    sT = st.Setup(N, shape, 0.2, 0.06, sa.transpose(0, 2, 1), ss.transpose(0, 2, 1))
    u = rng.normal(size=(16,) + shape)
    def S(v):
        vt = v.transpose(0, 1, 3, 2)
        return np.einsum("ij,j...->i...", T, vt)
    a = S(st.run(s, u, 3))
    b = st.run(sT, S(u), 3)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_translation_bitwise():
    s, u = _setup(3, (4, 5, 6), 31, q=True)
    shift = lambda v: np.roll(v, 1, axis=-2)
    s2 = st.Setup(3, (4, 5, 6), s.h[0], s.dt, np.roll(s.sigma_a, 1, axis=-2),
                  np.roll(s.sigma_s, 1, axis=-2), np.roll(s.q, 1, axis=-2))
    a = shift(st.run(s, u, 2))
    b = st.run(s2, shift(u), 2)
    assert np.array_equal(a, b)


# --------------------------------------------------------------- adjoint ---

def test_substep_dot_product():
    """<S w, v> = <w, S^T v> for the linear part of a substep (dense check of
    the transposed operator used by the adjoint)."""
    s, _ = _setup(3, (3, 4, 5), 40)
    rng = np.random.default_rng(41)
    for p, tau in ((1, 0.5 * s.dt), (0, s.dt)):
        A, _ = dense.substep_matrix(s, p, tau)
        w = rng.normal(size=A.shape[0])
        lam = rng.normal(size=A.shape[0]).reshape((s.V,) + s.shape)
        gc = np.zeros_like(lam)
        lt = adj.substep_T(s, np.zeros_like(lam), lam.copy(), p, tau, gc)
        assert abs((A @ w) @ lam.ravel() - w @ lt.ravel()) < 1e-12 * np.abs(w).sum()


def test_adjoint_gradient_vs_central_differences():
    N, shape = 3, (3, 4, 4)
    rng = np.random.default_rng(50)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=(16,) + shape)
    tgt = rng.normal(size=shape)
    h, dt, n = 0.25, 0.08, 4
    s = st.Setup(N, shape, h, dt, sa, ss, q)
    L, ga, gs, _ = adj.loss_and_grad(s, u, n, tgt)

    def loss(a, b):
        v = st.run(st.Setup(N, shape, h, dt, a, b, q), u, n)
        d = v[0] - tgt
        return 0.5 * np.sum(d * d)
    eps = 1e-5
    for c in [(0, 0, 0), (1, 2, 3), (2, 3, 1)]:
        e = np.zeros(shape)
        e[c] = eps
        fa = (loss(sa + e, ss) - loss(sa - e, ss)) / (2 * eps)
        fs = (loss(sa, ss + e) - loss(sa, ss - e)) / (2 * eps)
        assert abs(fa - ga[c]) < 1e-7 * max(1.0, abs(fa))
        assert abs(fs - gs[c]) < 1e-7 * max(1.0, abs(fs))


def test_dbeta_series_continuity():
    tau = 0.01
    c = np.array([0.0, 1e-6, 0.0999, 0.1001, 5.0])
    d = adj.dbeta_dc(c, tau)
    assert abs(d[0] + tau * tau / 2) < 1e-20
    ref = np.array([(st.E(-(cc + 1e-7) * tau) * tau - st.E(-(cc - 1e-7) * tau) * tau)[()] / 2e-7
                    for cc in c[1:]])
    assert np.allclose(d[1:], ref, rtol=1e-6)


def test_rectangular_cells_fourier_and_dense():
    """Rectangular dx x dy x dz cells (Sec. 2.1): the array stepping agrees with
    the dense assembly and a plane wave evolves by the symbol with per-direction
    difference symbols 2 i sin(k_d h_d / 2) / h_d."""
    N, shape = 3, (5, 4, 6)
    h = (1.0 / 6, 1.0 / 4 * 0.7, 1.0 / 5 * 1.3)
    dt = 0.3 * min(h)
    rng = np.random.default_rng(60)
    sa = np.full(shape, 0.25)
    ss = np.full(shape, 0.6)
    s = st.Setup(N, shape, h, dt, sa, ss)
    L = (shape[2] * h[0], shape[1] * h[1], shape[0] * h[2])
    k = 2 * np.pi * np.array([1.0 / L[0], -1.0 / L[1], 2.0 / L[2]])
    uh = rng.normal(size=16) + 1j * rng.normal(size=16)
    ph = np.empty((16,) + shape, dtype=complex)
    for i in range(16):
        x, y, z = dense.staggered_positions(shape, h, s.o[i])
        ph[i] = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    G = dense.fourier_symbol(N, k, h, dt, 0.25, 0.85)
    want = ((np.linalg.matrix_power(G, 4) @ uh)[:, None, None, None] * ph).real
    assert np.abs(st.run(s, (uh[:, None, None, None] * ph).real, 4) - want).max() < 1e-13 * np.abs(want).max()
    sr = st.Setup(N, shape, h, dt, rng.uniform(0, .5, shape), rng.uniform(0, 1, shape), rng.uniform(0, 1, shape))
    u = rng.normal(size=(16,) + shape)
    S, b = dense.step_matrix(sr)
    x = u.ravel().copy()
    for _ in range(2):
        x = S @ x + b
    assert np.abs(x - st.run(sr, u, 2).ravel()).max() <= 1e-13 * np.abs(x).max()


def test_cfl_limit_rectangular_cells():
    """sigma = 0 with unequal edges: stable iff dt <= 1/(lambda_max sqrt(sum 1/h_d^2))."""
    N = 3
    h = (1.0, 0.6, 1.7)
    lam = np.polynomial.legendre.leggauss(N + 1)[0].max()
    lim = 1.0 / (lam * np.sqrt(sum(1.0 / v ** 2 for v in h)))
    ks = np.linspace(0, np.pi, 5)
    def radius(dt):
        r = 0.0
        for a in ks:
            for b in ks:
                for c in ks:
                    kv = (a / h[0], b / h[1], c / h[2])
                    G = dense.fourier_symbol(N, kv, h, dt, 0.0, 0.0)
                    r = max(r, np.abs(np.linalg.eigvals(G)).max())
        return r
    assert radius(0.98 * lim) <= 1 + 1e-10
    assert radius(1.05 * lim) > 1 + 1e-6


# ------------------------------------------------- anisotropic scattering ---
# Sec. 2 (moment equations): the collision coefficient of degree l is
# Sigma_a + Sigma_s0 - Sigma_sl.  The oracle takes Sigma_sl = g_l sigma_s.

def _scattering_matrix(N, g):
    """int int R_i(W) p(W.W') R_j(W') dW dW' by quadrature for the phase
    function p(m) = sum_l (2l+1)/(4 pi) g_l P_l(m) (degree <= N)."""
    mu, phi, w = basis.sphere_rule(N, extra=2)
    R = basis.real_sh(N, mu, phi)
    X = np.stack(basis.directions(mu, phi))
    cosg = np.clip(X.T @ X, -1.0, 1.0)
    p = np.zeros_like(cosg)
    for l, gl in enumerate(g):
        p += (2 * l + 1) / (4 * np.pi) * gl * np.polynomial.legendre.Legendre.basis(l)(cosg)
    return (R * w) @ p @ (R * w).T


def test_scattering_operator_diagonal_per_degree():
    """A kernel depending only on the angle between directions is diagonal
    in the real harmonics, with the Legendre moment g_l on degree l
    (Funk-Hecke): the reading behind c_l = sigma_a + (1 - g_l) sigma_s."""
    N = 4
    g = [1.0, 0.55, -0.2, 0.3, 0.1]
    S = _scattering_matrix(N, g)
    ell = np.array([basis.lm_of(i)[0] for i in range(basis.n_moments(N))])
    assert np.abs(S - np.diag(np.array(g)[ell])).max() < 1e-13


def test_anisotropic_homogeneous_decay_from_quadrature():
    """Homogeneous state and medium: moment i decays as exp(-c_i t) with
    c_i = sigma_a + sigma_s - sigma_s S_ii, S from the angular quadrature
    of the phase function (not from the oracle's formula)."""
    N, shape = 3, (3, 3, 3)
    sa, ss = 0.4, 1.1
    g = [1.0, 0.7, 0.35, -0.25]
    S = _scattering_matrix(N, g)
    c = sa + ss - ss * np.diag(S)
    s = st.Setup(N, shape, 0.2, 0.05, np.full(shape, sa), np.full(shape, ss), scattering=g[1:])
    u0 = np.arange(1.0, 17.0)[:, None, None, None] * np.ones((16,) + shape)
    v = u0.copy()
    for k in range(1, 9):
        st.step(s, v)
        want = u0[:, 0, 0, 0] * np.exp(-c * k * s.dt)
        assert np.abs(v[:, 0, 0, 0] - want).max() < 1e-14 * 16
        assert np.abs(v - v[:, :1, :1, :1]).max() == 0.0


def test_anisotropic_fourier_mode():
    """Plane wave on a homogeneous medium with per-degree coefficients:
    the Strang product of the substep symbols with c_l on degree l."""
    N, shape = 3, (6, 6, 6)
    h = 1.0 / 6
    dt = 0.4 * h
    sa, ss = 0.2, 0.9
    g = [0.6, 0.36, 0.216]
    s = st.Setup(N, shape, h, dt, np.full(shape, sa), np.full(shape, ss), scattering=g)
    c_deg = [sa] + [sa + (1 - gl) * ss for gl in g]
    k = 2 * np.pi * np.array([1.0, -2.0, 1.0])
    rng = np.random.default_rng(70)
    uh = rng.normal(size=s.V) + 1j * rng.normal(size=s.V)
    ph = np.empty((s.V,) + shape, dtype=complex)
    for i in range(s.V):
        x, y, z = dense.staggered_positions(shape, (h, h, h), s.o[i])
        ph[i] = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    G = dense.fourier_symbol(N, k, (h, h, h), dt, 0, 0, c_deg=c_deg)
    want = ((np.linalg.matrix_power(G, 5) @ uh)[:, None, None, None] * ph).real
    got = st.run(s, (uh[:, None, None, None] * ph).real, 5)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_anisotropic_conservation_and_isotropic_limit():
    """g_0 = 1 keeps sum u_0 constant for sigma_a = 0, q = 0 whatever g_l;
    g_l = 0 is the isotropic scheme bit for bit."""
    shape = (4, 5, 3)
    rng = np.random.default_rng(71)
    ss = rng.uniform(0, 1, shape)
    u = rng.normal(size=(16,) + shape)
    s = st.Setup(3, shape, 0.25, 0.08, np.zeros(shape), ss, scattering=[0.9, -0.5, 0.3])
    v = u.copy()
    for _ in range(10):
        st.step(s, v)
    assert abs(v[0].sum() - u[0].sum()) < 1e-14 * np.abs(u[0]).sum()
    sa = rng.uniform(0, 0.5, shape)
    a = st.run(st.Setup(3, shape, 0.25, 0.08, sa, ss), u, 3)
    b = st.run(st.Setup(3, shape, 0.25, 0.08, sa, ss, scattering=[0.0, 0.0, 0.0]), u, 3)
    assert np.array_equal(a, b)


def test_anisotropic_dense_and_contractive():
    """Dense assembly equals the array stepping with per-degree
    coefficients, and the step stays contractive below the CFL limit."""
    rng = np.random.default_rng(72)
    shape = (3, 4, 4)
    s = st.Setup(3, shape, 0.25, 0.1, rng.uniform(0, .5, shape), rng.uniform(0, 1, shape),
                 rng.uniform(0, 1, shape), scattering=[0.8, 0.5, -0.4])
    u = rng.normal(size=(16,) + shape)
    S, b = dense.step_matrix(s)
    x = u.ravel().copy()
    for _ in range(3):
        x = S @ x + b
    assert np.abs(x - st.run(s, u, 3).ravel()).max() <= 1e-13 * np.abs(x).max()
    assert np.abs(np.linalg.eigvals(S.toarray())).max() <= 1 + 1e-12


def test_anisotropic_adjoint_vs_central_differences():
    N, shape = 3, (3, 3, 4)
    rng = np.random.default_rng(73)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    g = [0.75, 0.4, -0.3]
    u = rng.normal(size=(16,) + shape)
    tgt = rng.normal(size=shape)
    h, dt, n = 0.25, 0.08, 3
    L, ga, gs, _ = adj.loss_and_grad(st.Setup(N, shape, h, dt, sa, ss, q, scattering=g), u, n, tgt)

    def loss(a, b):
        v = st.run(st.Setup(N, shape, h, dt, a, b, q, scattering=g), u, n)
        d = v[0] - tgt
        return 0.5 * np.sum(d * d)
    eps = 1e-5
    for c in [(0, 0, 0), (1, 2, 3), (2, 1, 0)]:
        e = np.zeros(shape)
        e[c] = eps
        fa = (loss(sa + e, ss) - loss(sa - e, ss)) / (2 * eps)
        fs = (loss(sa, ss + e) - loss(sa, ss - e)) / (2 * eps)
        assert abs(fa - ga[c]) < 1e-7 * max(1.0, abs(fa))
        assert abs(fs - gs[c]) < 1e-7 * max(1.0, abs(fs))
