"""Oracle (test infrastructure only): ctypes front end of pn_oracle.c.

The flux matrices and parities handed to the C code come from oracle.basis
(quadrature and evaluated reflections), never from the product library.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import basis
from .stepper import scattering_moments

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pn_oracle.c")
_LIB = os.path.join(_HERE, "libpn_oracle.so")
_lib = None


def build(force=True):
    """Compile the C oracle (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i32, f64 = ctypes.c_int, ctypes.c_double
        common = [i32, i32, i32, i32, f64, f64, f64, f64, P(i32), i32, P(i32), P(i32), P(i32),
                  P(f64), P(f64), P(f64), P(f64), P(f64)]
        L.pno_run.argtypes = common + [P(f64), i32, i32]
        L.pno_run.restype = i32
        L.pno_grad.argtypes = common + [P(f64), i32, i32, P(f64), P(f64), P(f64), i32]
        L.pno_grad.restype = f64
        L.pno_threads.restype = i32
        _lib = L
    return _lib


class Tables:
    """Flux-matrix triples and parities for one N (computed once per N)."""
    _cache = {}

    def __new__(cls, N):
        if N in cls._cache:
            return cls._cache[N]
        self = super().__new__(cls)
        M = basis.flux_matrices(N)
        ti, sj, dr, vv = [], [], [], []
        for d in range(3):
            ii, jj = np.nonzero(M[d])
            ti.append(ii); sj.append(jj); dr.append(np.full(ii.size, d)); vv.append(M[d][ii, jj])
        self.N = N
        self.V = basis.n_moments(N)
        self.ti = np.ascontiguousarray(np.concatenate(ti), dtype=np.int32)
        self.sj = np.ascontiguousarray(np.concatenate(sj), dtype=np.int32)
        self.dr = np.ascontiguousarray(np.concatenate(dr), dtype=np.int32)
        self.vv = np.ascontiguousarray(np.concatenate(vv), dtype=np.float64)
        self.o = np.ascontiguousarray(basis.reflection_parities(N), dtype=np.int32)
        cls._cache[N] = self
        return self


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _args(T, shape, h, dt, sa, ss, q, scattering=None):
    nz, ny, nx = shape
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    i32, f64 = ctypes.c_int, ctypes.c_double
    sa = np.ascontiguousarray(sa, dtype=np.float64).reshape(-1)
    ss = np.ascontiguousarray(ss, dtype=np.float64).reshape(-1)
    q = (np.zeros(nx * ny * nz) if q is None
         else np.ascontiguousarray(q, dtype=np.float64).reshape(-1))
    gl = None if scattering is None else np.ascontiguousarray(scattering_moments(T.N, scattering))
    keep = (sa, ss, q, gl)
    return keep, [T.V, nx, ny, nz, hx, hy, hz, dt, _p(T.o, i32), int(T.ti.size), _p(T.ti, i32),
                  _p(T.sj, i32), _p(T.dr, i32), _p(T.vv, f64), _p(sa, f64), _p(ss, f64), _p(q, f64),
                  None if gl is None else _p(gl, f64)]


def run(N, shape, h, dt, sa, ss, q, u0, nsteps, threads=0, scattering=None):
    """Moments after nsteps literal Strang steps; u0 of shape (V, nz, ny, nx).
    scattering: g_l for l = 1, 2, ... (None: isotropic)."""
    T = Tables(N)
    u = np.array(u0, dtype=np.float64, order="C", copy=True).reshape((T.V,) + tuple(shape))
    keep, a = _args(T, shape, h, dt, sa, ss, q, scattering)
    lib().pno_run(*a, _p(u, ctypes.c_double), int(nsteps), int(threads))
    del keep
    return u


def grad(N, shape, h, dt, sa, ss, q, u0, nsteps, ck, target, threads=0, scattering=None):
    """(L, dL/dsigma_a, dL/dsigma_s) for L = 1/2 ||u_0(T) - target||^2."""
    T = Tables(N)
    u = np.ascontiguousarray(u0, dtype=np.float64).reshape((T.V,) + tuple(shape))
    tg = np.ascontiguousarray(target, dtype=np.float64).reshape(-1)
    dsa = np.zeros(tg.size)
    dss = np.zeros(tg.size)
    keep, a = _args(T, shape, h, dt, sa, ss, q, scattering)
    L = lib().pno_grad(*a, _p(u, ctypes.c_double), int(nsteps), int(ck), _p(tg, ctypes.c_double),
                       _p(dsa, ctypes.c_double), _p(dss, ctypes.c_double), int(threads))
    del keep
    return L, dsa.reshape(shape), dss.reshape(shape)


def threads():
    return int(lib().pno_threads())
