"""Pins of the C/OpenMP oracle: it must reproduce the numpy oracle (itself
pinned in test_oracle_pins.py) and the closed-form facts directly."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import c_oracle as co
from oracle import dense
from oracle import stepper as st


@pytest.fixture(scope="module", autouse=True)
def built():
    co.build(force=False)


@pytest.mark.parametrize("N,shape", [(3, (4, 5, 6)), (2, (1, 1, 7)), (7, (3, 3, 3)), (1, (2, 1, 3))])
def test_c_matches_numpy(N, shape):
    rng = np.random.default_rng(N)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    s = st.Setup(N, shape, 0.2, 0.07, sa, ss, q)
    u = rng.normal(size=(s.V,) + shape)
    a = st.run(s, u, 4)
    b = co.run(N, shape, 0.2, 0.07, sa, ss, q, u, 4)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(a).max() * 4


def test_c_fourier_mode():
    N, shape = 3, (8, 8, 8)
    h = 1.0 / 8
    dt = 0.45 * h
    s = st.Setup(N, shape, h, dt, np.full(shape, 0.2), np.full(shape, 0.5))
    k = 2 * np.pi * np.array([1.0, -2.0, 3.0])
    rng = np.random.default_rng(3)
    uh = rng.normal(size=16) + 1j * rng.normal(size=16)
    ph = np.empty((16,) + shape, dtype=complex)
    for i in range(16):
        x, y, z = dense.staggered_positions(shape, (h, h, h), s.o[i])
        ph[i] = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    G = dense.fourier_symbol(N, k, (h, h, h), dt, 0.2, 0.7)
    want = ((np.linalg.matrix_power(G, 6) @ uh)[:, None, None, None] * ph).real
    got = co.run(N, shape, h, dt, np.full(shape, 0.2), np.full(shape, 0.5), None,
                 (uh[:, None, None, None] * ph).real, 6)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_c_conservation_P7():
    shape = (8, 9, 10)
    rng = np.random.default_rng(5)
    u = rng.normal(size=(64,) + shape)
    got = co.run(7, shape, 0.1, 0.05, np.zeros(shape), rng.uniform(0, 2, shape), None, u, 10)
    assert abs(got[0].sum() - u[0].sum()) < 1e-13 * np.abs(u[0]).sum()


def test_c_adjoint_matches_numpy():
    N, shape = 3, (3, 4, 5)
    rng = np.random.default_rng(6)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=(16,) + shape)
    tgt = rng.normal(size=shape)
    s = st.Setup(N, shape, 0.2, 0.07, sa, ss, q)
    L, ga, gs, _ = adj.loss_and_grad(s, u, 7, tgt)
    for ck in (1, 3, 7, 10):
        L2, ga2, gs2 = co.grad(N, shape, 0.2, 0.07, sa, ss, q, u, 7, ck, tgt)
        assert abs(L - L2) < 1e-14 * L
        assert np.abs(ga - ga2).max() < 1e-13 * np.abs(ga).max()
        assert np.abs(gs - gs2).max() < 1e-13 * np.abs(gs).max()


@pytest.mark.parametrize("N,shape", [(3, (4, 5, 6)), (7, (3, 4, 3))])
def test_c_anisotropic_matches_numpy(N, shape):
    """Per-degree scattering moments: forward and adjoint of the C oracle
    against the numpy oracle."""
    rng = np.random.default_rng(20 + N)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    g = [0.6 ** l for l in range(1, N + 1)]
    s = st.Setup(N, shape, 0.2, 0.07, sa, ss, q, scattering=g)
    u = rng.normal(size=(s.V,) + shape)
    a = st.run(s, u, 3)
    b = co.run(N, shape, 0.2, 0.07, sa, ss, q, u, 3, scattering=g)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(a).max() * 4
    tgt = rng.normal(size=shape)
    L1, ga1, gs1, _ = adj.loss_and_grad(s, u, 3, tgt)
    L2, ga2, gs2 = co.grad(N, shape, 0.2, 0.07, sa, ss, q, u, 3, 2, tgt, scattering=g)
    assert abs(L1 - L2) <= 1e-14 * abs(L1)
    assert np.abs(ga1 - ga2).max() <= 1e-13 * np.abs(ga1).max()
    assert np.abs(gs1 - gs2).max() <= 1e-13 * np.abs(gs1).max()
