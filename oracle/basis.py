"""Oracle (test infrastructure only): angular basis and flux matrices.

Follows Sec. 2 of Berghoff, Frank, Seibold (arXiv 2004.02833):
  * moments psi_l^m are projections on spherical harmonics (Sec. 2, the text
    after eq. (2)); a real basis is obtained by taking the real and imaginary
    parts of the complex harmonics Y_l^m (the "appropriate substitutions");
  * the 3D moment system is eq. (3) with symmetric flux matrices M_x, M_y, M_z
    whose entries the paper does not print.

Reading used here (orthonormal real harmonics, z polar axis):
  R_{l,0}  = Y_l^0
  R_{l,m}  = sqrt(2) (-1)^m Re Y_l^m   (m > 0)
  R_{l,-m} = sqrt(2) (-1)^m Im Y_l^m   (m > 0)
with Y_l^m the complex harmonic including the (-1)^m phase as written in the
paper.  The (-1)^m cancels that phase, so R_{l,m} = sqrt(2) N_l^m P_l^m cos(m phi)
with P_l^m free of the Condon-Shortley sign.  Y_l^m is taken from
scipy.special.sph_harm_y (a library primitive).

M_d[i, j] = integral over the sphere of Omega_d R_i R_j, evaluated by a product
rule (Gauss-Legendre in mu = cos(theta), uniform in phi) that is exact for the
polynomial degrees involved.  The moment index is i = l^2 + l + m.
"""
import numpy as np
from scipy.special import sph_harm_y

FAMILY_ORDER = ("G111", "G221", "G212", "G122", "G211", "G121", "G112", "G222")
"""Storage order of the eight sub-grids (Sec. 3.2, "Reorder components")."""


def n_moments(N):
    return (N + 1) * (N + 1)


def moment_index(l, m):
    return l * l + l + m


def lm_of(i):
    l = int(np.floor(np.sqrt(i) + 1e-12))
    while (l + 1) * (l + 1) <= i:
        l += 1
    while l * l > i:
        l -= 1
    return l, i - l * l - l


def real_sh(N, mu, phi):
    """Real orthonormal harmonics R_i(mu, phi) for l <= N; shape (V, npts)."""
    mu = np.asarray(mu, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    theta = np.arccos(np.clip(mu, -1.0, 1.0))
    R = np.empty((n_moments(N),) + mu.shape)
    for l in range(N + 1):
        R[moment_index(l, 0)] = sph_harm_y(l, 0, theta, phi).real
        for m in range(1, l + 1):
            Y = sph_harm_y(l, m, theta, phi)
            s = np.sqrt(2.0) * (-1.0) ** m
            R[moment_index(l, m)] = s * Y.real
            R[moment_index(l, -m)] = s * Y.imag
    return R


def sphere_rule(N, extra=2):
    """Product quadrature on S^2: Gauss-Legendre in mu, uniform in phi.

    With n_mu = N + extra nodes it integrates polynomials in mu of degree
    2 N + 2 extra - 1 exactly; n_phi = 2 N + 2 extra points integrate the
    trigonometric products up to frequency 2 N + 2 extra - 1 exactly.  The
    integrands Omega_d R_i R_j have degree at most 2 N + 1.
    Returns (mu, phi, w) flattened; sum(w) = 4 pi.
    """
    n_mu = N + extra
    n_phi = 2 * N + 2 * extra
    x, wx = np.polynomial.legendre.leggauss(n_mu)
    ph = 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    MU, PH = np.meshgrid(x, ph, indexing="ij")
    W = np.outer(wx, np.full(n_phi, 2.0 * np.pi / n_phi))
    return MU.ravel(), PH.ravel(), W.ravel()


def directions(mu, phi):
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return s * np.cos(phi), s * np.sin(phi), mu


def gauss_legendre_ld(n):
    """Gauss-Legendre nodes/weights on [-1, 1] in long double.

    Double-precision nodes from numpy are polished by Newton steps on P_n,
    evaluated with the three-term recurrence in 80-bit arithmetic.
    """
    x0, _ = np.polynomial.legendre.leggauss(n)
    x = x0.astype(np.longdouble)
    for _ in range(4):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = n * (x * p1 - p0) / (x * x - 1)
        x = x - p1 / dp
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    w = 2 / ((1 - x * x) * dp * dp)
    return x, w


def polar_factors(N, mu):
    """Theta_{l,|m|}(mu) with R_{l,m} = Theta_{l,|m|}(mu) * Phi_m(phi), long double.

    Theta_{l,0} = N_l^0 P_l,  Theta_{l,m} = sqrt(2) N_l^m P_l^m (m >= 1), where
    P_l^m carries no Condon-Shortley sign and
    N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  P_l^m is evaluated by the
    textbook recurrences P_m^m = (2m-1)!! (1-mu^2)^(m/2),
    P_{m+1}^m = (2m+1) mu P_m^m, (l-m) P_l^m = (2l-1) mu P_{l-1}^m - (l+m-1) P_{l-2}^m.
    Returns a dict (l, m>=0) -> values.
    """
    mu = np.asarray(mu, dtype=np.longdouble)
    s = np.sqrt(1 - mu * mu)
    out = {}
    pmm = np.ones_like(mu)
    for m in range(N + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        fac = np.longdouble(1)
        prev2, prev1 = None, pmm
        for l in range(m, N + 1):
            if l == m + 1:
                cur = (2 * m + 1) * mu * pmm
            elif l >= m + 2:
                cur = ((2 * l - 1) * mu * prev1 - (l + m - 1) * prev2) / (l - m)
            else:
                cur = pmm
            if l > m:
                prev2, prev1 = prev1, cur
            # (l-m)!/(l+m)! as a product, in long double
            r = np.longdouble(1)
            for k in range(l - m + 1, l + m + 1):
                r /= k
            norm = np.sqrt((2 * l + 1) / (4 * np.pi * np.longdouble(1)) * r)
            if m > 0:
                norm = norm * np.sqrt(np.longdouble(2))
            out[(l, m)] = norm * cur
    return out


def azimuthal_factor(m, phi):
    phi = np.asarray(phi, dtype=np.longdouble)
    if m > 0:
        return np.cos(m * phi)
    if m < 0:
        return np.sin(-m * phi)
    return np.ones_like(phi)


def flux_matrices(N, tol=1e-14):
    """(M_x, M_y, M_z) of eq. (3), dense (V, V); |entries| < tol set to 0.

    M_d[i, j] = integral of Omega_d R_i R_j over the sphere.  With
    Omega_x = sqrt(1-mu^2) cos(phi), Omega_y = sqrt(1-mu^2) sin(phi),
    Omega_z = mu and R_i = Theta_i(mu) Phi_i(phi) the integral is a product of
    a mu-integral (Gauss-Legendre, N + 2 nodes, exact for the polynomial
    integrands that occur) and a phi-integral (uniform rule with 2N + 4 points,
    exact for the trigonometric products).  Everything runs in long double and
    is rounded to double at the end.
    """
    V = n_moments(N)
    x, wx = gauss_legendre_ld(N + 2)
    n_phi = 2 * N + 4
    ph = 2 * np.pi * (np.arange(n_phi, dtype=np.longdouble) + np.longdouble(0.5)) / n_phi
    wph = np.full(n_phi, 2 * np.pi * np.longdouble(1) / n_phi)
    th = polar_factors(N, x)
    keys = sorted(th)                       # unique (l, |m|)
    kpos = {k: a for a, k in enumerate(keys)}
    T = np.stack([th[k] for k in keys])     # (n_lm, n_mu)
    ms = list(range(-N, N + 1))
    F = np.stack([azimuthal_factor(m, ph) for m in ms])   # (2N+1, n_phi)
    sx = np.sqrt(1 - x * x)
    A_sin = (T * (wx * sx)) @ T.T           # mu-integral with sqrt(1-mu^2)
    A_mu = (T * (wx * x)) @ T.T             # mu-integral with mu
    B_one = (F * wph) @ F.T
    B_cos = (F * (wph * np.cos(ph))) @ F.T
    B_sin = (F * (wph * np.sin(ph))) @ F.T
    li = np.empty(V, dtype=np.int64)
    mi = np.empty(V, dtype=np.int64)
    for i in range(V):
        l, m = lm_of(i)
        li[i] = kpos[(l, abs(m))]
        mi[i] = m + N
    out = []
    for A, B in ((A_sin, B_cos), (A_sin, B_sin), (A_mu, B_one)):
        M = (A[np.ix_(li, li)] * B[np.ix_(mi, mi)]).astype(np.float64)
        M[np.abs(M) < tol] = 0.0
        out.append(M)
    return tuple(out)


def gram_matrix(N):
    """Integral of R_i R_j over the sphere with scipy's harmonics (double)."""
    mu, phi, w = sphere_rule(N)
    R = real_sh(N, mu, phi)
    return (R * w) @ R.T


def separable_sh(N, mu, phi):
    """R_i(mu, phi) = Theta_i(mu) Phi_i(phi) from polar_factors (long double)."""
    th = polar_factors(N, mu)
    V = n_moments(N)
    R = np.empty((V,) + np.shape(mu), dtype=np.longdouble)
    for i in range(V):
        l, m = lm_of(i)
        R[i] = th[(l, abs(m))] * azimuthal_factor(m, phi)
    return R


def reflection_parities(N, seed=12345):
    """o[i] = (o_x, o_y, o_z): o_d = 1 iff R_i is odd under Omega_d -> -Omega_d.

    Decided numerically by evaluating the basis at random directions and at
    their reflections (Sec. 2.1: a derivative in d maps a (1,.,.) grid to a
    (2,.,.) grid; the moment on G_{1+o_x,1+o_y,1+o_z}).
    """
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, 16))
    v /= np.linalg.norm(v, axis=0)
    V = n_moments(N)
    o = np.zeros((V, 3), dtype=np.int64)

    def ev(x, y, z):
        return real_sh(N, z, np.arctan2(y, x))

    base = ev(*v)
    for d in range(3):
        r = v.copy()
        r[d] = -r[d]
        refl = ev(*r)
        for i in range(V):
            scale = np.max(np.abs(base[i]))
            if np.allclose(refl[i], -base[i], atol=1e-12 * scale):
                o[i, d] = 1
            elif np.allclose(refl[i], base[i], atol=1e-12 * scale):
                o[i, d] = 0
            else:
                raise AssertionError("basis function %d has no parity in %d" % (i, d))
    return o


def family_name(o):
    return "G%d%d%d" % (1 + o[0], 1 + o[1], 1 + o[2])


def families(N):
    """List of sub-grid names per moment, e.g. 'G111' for moment 0."""
    return [family_name(oi) for oi in reflection_parities(N)]
