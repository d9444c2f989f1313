"""Thin ctypes binding of libpm (the C ABI in include/pm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Host arrays are numpy float64 in [z, y, x] order (x fastest);
device pointers are plain integers (e.g. torch's tensor.data_ptr()).
Raises PmError for any negative return code.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpm.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EDEVICE, PM_ESTATE, PM_ENONFINITE = 0, -1, -2, -3, -4, -5
PM_FP64, PM_FP32, PM_BF16 = 0, 1, 2
PM_N_MAX = 63

EXPORTED = ("pm_set_precision", "pm_set_scattering", "pm_init", "pm_init_cells", "pm_write", "pm_write_dev", "pm_step", "pm_set_merge",
            "pm_read",
            "pm_read_dev", "pm_set_checkpoint", "pm_grad", "pm_grad_dev", "pm_recording_id",
            "pm_total", "pm_check", "pm_check_noalloc",
            "pm_bind_stream", "pm_sync", "pm_cfl_warning", "pm_timing", "pm_sweep_times",
            "pm_finalize", "pm_last_error", "pm_flux_nnz", "pm_flux_entries", "pm_moment_grid",
            "pm_moment_slot", "pm_halo_plan", "pm_halo_pack", "pm_halo_unpack", "pm_device_bytes")


class PmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libpm error %d: %s" % (code, msg))
        self.code = code


_lib = None
_shape = None       # (nz, ny, nx) of the live context
_V = 0


def lib():
    """Load libpm.so; fails loudly if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpm.so not found at %s: build it with "
                               "`python -m paper_2004_02833_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        i32, f64, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        sig = {
            "pm_set_precision": ([i32], i32),
            "pm_set_scattering": ([P(f64), i32], i32),
            "pm_init": ([i32, i32, i32, i32, f64, f64, P(f64), P(f64), P(f64)], i32),
            "pm_init_cells": ([i32, i32, i32, i32, f64, f64, f64, f64, P(f64), P(f64), P(f64)], i32),
            "pm_write": ([i32, P(f64)], i32),
            "pm_write_dev": ([i32, vp], i32),
            "pm_step": ([i32], i32),
            "pm_set_merge": ([i32], i32),
            "pm_read": ([i32, P(f64)], i32),
            "pm_read_dev": ([i32, vp], i32),
            "pm_set_checkpoint": ([i32], i32),
            "pm_grad": ([P(f64), P(f64), P(f64)], i32),
            "pm_grad_dev": ([vp, vp, vp], i32),
            "pm_recording_id": ([], i64),
            "pm_total": ([P(f64)], i32),
            "pm_check": ([P(f64), P(i64)], i32),
            "pm_check_noalloc": ([vp, vp], i32),
            "pm_bind_stream": ([vp], i32),
            "pm_sync": ([], i32),
            "pm_cfl_warning": ([], i32),
            "pm_timing": ([i32], i32),
            "pm_sweep_times": ([P(i32), P(f64), P(i32), P(f64)], i32),
            "pm_finalize": ([], None),
            "pm_last_error": ([], ctypes.c_char_p),
            "pm_flux_nnz": ([i32], i32),
            "pm_flux_entries": ([i32, P(i32), P(i32), P(i32), P(f64), i32], i32),
            "pm_moment_grid": ([i32, i32], i32),
            "pm_moment_slot": ([i32, i32], i32),
            "pm_halo_plan": ([i32, i32, i32, i32, i32, i32, P(i64), P(i64), i64], i64),
            "pm_halo_pack": ([i32, i32, vp], i32),
            "pm_halo_unpack": ([i32, i32, vp], i32),
            "pm_device_bytes": ([], i64),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise PmError(rc, pm_last_error())
    return rc


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(a, n, name):
    arr = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if arr.size != n:
        raise ValueError("%s has %d values, expected %d" % (name, arr.size, n))
    return arr


def pm_last_error():
    return lib().pm_last_error().decode()


def pm_set_precision(precision):
    return _check(lib().pm_set_precision(int(precision)))


def pm_set_scattering(g=None):
    """Per-degree scattering moments g_1, g_2, ... for the next pm_init
    (None or empty: isotropic)."""
    if g is None or len(g) == 0:
        return _check(lib().pm_set_scattering(None, 0))
    arr = np.ascontiguousarray(np.asarray(g, dtype=np.float64).ravel())
    return _check(lib().pm_set_scattering(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          int(arr.size)))


def pm_init(N, nx, ny, nz, dx, dt, sigma_a, sigma_s, q=None):
    global _shape, _V
    n = int(nx) * int(ny) * int(nz)
    if min(int(nx), int(ny), int(nz)) < 1:
        n = -1          # let the library report the invalid grid
    fld = (lambda a, name: _field(a, n, name)) if n > 0 else (
        lambda a, name: np.ascontiguousarray(a, dtype=np.float64).reshape(-1))
    sa = fld(sigma_a, "sigma_a")
    ss = fld(sigma_s, "sigma_s")
    qq = None if q is None else fld(q, "q")
    rc = lib().pm_init(int(N), int(nx), int(ny), int(nz), float(dx), float(dt), _dptr(sa),
                       _dptr(ss), None if qq is None else _dptr(qq))
    _check(rc)
    _shape = (int(nz), int(ny), int(nx))
    _V = (int(N) + 1) ** 2
    return rc


def pm_init_cells(N, nx, ny, nz, dx, dy, dz, dt, sigma_a, sigma_s, q=None):
    """pm_init for rectangular dx x dy x dz cells."""
    global _shape, _V
    n = int(nx) * int(ny) * int(nz)
    if min(int(nx), int(ny), int(nz)) < 1:
        n = -1
    fld = (lambda a, name: _field(a, n, name)) if n > 0 else (
        lambda a, name: np.ascontiguousarray(a, dtype=np.float64).reshape(-1))
    sa = fld(sigma_a, "sigma_a")
    ss = fld(sigma_s, "sigma_s")
    qq = None if q is None else fld(q, "q")
    rc = lib().pm_init_cells(int(N), int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                             float(dt), _dptr(sa), _dptr(ss), None if qq is None else _dptr(qq))
    _check(rc)
    _shape = (int(nz), int(ny), int(nx))
    _V = (int(N) + 1) ** 2
    return rc


def _need_ctx():
    if _shape is None:
        raise PmError(PM_ESTATE, "no context: call pm_init first")
    return _shape


def pm_write(moment, src):
    shape = _need_ctx()
    a = _field(src, int(np.prod(shape)), "src")
    return _check(lib().pm_write(int(moment), _dptr(a)))


def pm_write_dev(moment, device_ptr):
    return _check(lib().pm_write_dev(int(moment), ctypes.c_void_p(int(device_ptr))))


def pm_step(nsteps):
    return _check(lib().pm_step(int(nsteps)))


def pm_set_merge(on):
    return _check(lib().pm_set_merge(int(on)))


def pm_read(moment, out=None):
    shape = _need_ctx()
    if out is None:
        out = np.empty(shape, dtype=np.float64)
    if out.dtype != np.float64 or not out.flags.c_contiguous or out.size != np.prod(shape):
        raise ValueError("out must be a C-contiguous float64 array of %s" % (shape,))
    _check(lib().pm_read(int(moment), _dptr(out)))
    return out


def pm_read_dev(moment, device_ptr):
    return _check(lib().pm_read_dev(int(moment), ctypes.c_void_p(int(device_ptr))))


def pm_set_checkpoint(k):
    return _check(lib().pm_set_checkpoint(int(k)))


def pm_grad(dL_du0):
    shape = _need_ctx()
    n = int(np.prod(shape))
    g = _field(dL_du0, n, "dL_du0")
    dsa = np.empty(shape)
    dss = np.empty(shape)
    _check(lib().pm_grad(_dptr(g), _dptr(dsa), _dptr(dss)))
    return dsa, dss


def pm_grad_dev(dL_du0_ptr, dsigma_a_ptr, dsigma_s_ptr):
    """Device-pointer form of pm_grad (integers, e.g. tensor.data_ptr();
    0 for an output that is not wanted)."""
    vp = lambda p: ctypes.c_void_p(int(p)) if p else None
    return _check(lib().pm_grad_dev(vp(dL_du0_ptr), vp(dsigma_a_ptr), vp(dsigma_s_ptr)))


def pm_recording_id():
    return int(lib().pm_recording_id())


def pm_total():
    v = ctypes.c_double()
    _check(lib().pm_total(ctypes.byref(v)))
    return v.value


def pm_check():
    """(max |u|, number of non-finite values); no exception for non-finite."""
    m = ctypes.c_double()
    k = ctypes.c_longlong()
    rc = lib().pm_check(ctypes.byref(m), ctypes.byref(k))
    if rc < 0 and rc != PM_ENONFINITE:
        _check(rc)
    return m.value, k.value


def pm_check_noalloc(dev_max_abs_ptr, dev_nonfinite_ptr):
    """pm_check into device memory (float64 max |u|, uint64 count) without
    allocation or synchronisation."""
    return _check(lib().pm_check_noalloc(ctypes.c_void_p(int(dev_max_abs_ptr)),
                                         ctypes.c_void_p(int(dev_nonfinite_ptr))))


def pm_bind_stream(stream_ptr):
    return _check(lib().pm_bind_stream(ctypes.c_void_p(int(stream_ptr) if stream_ptr else 0)))


def pm_sync():
    return _check(lib().pm_sync())


def pm_cfl_warning():
    return int(lib().pm_cfl_warning())


def pm_timing(on):
    return _check(lib().pm_timing(1 if on else 0))


def pm_sweep_times():
    no, ne = ctypes.c_int(), ctypes.c_int()
    to, te = ctypes.c_double(), ctypes.c_double()
    _check(lib().pm_sweep_times(ctypes.byref(no), ctypes.byref(to), ctypes.byref(ne),
                                ctypes.byref(te)))
    return {"odd": (no.value, to.value), "even": (ne.value, te.value)}


def pm_finalize():
    global _shape, _V
    lib().pm_finalize()
    _shape = None
    _V = 0


def pm_flux_nnz(N):
    return _check(lib().pm_flux_nnz(int(N)))


def pm_flux_entries(N):
    """(row, col, dir, value) arrays of the closed-form M_x, M_y, M_z."""
    n = pm_flux_nnz(N)
    r = np.empty(n, np.int32)
    c = np.empty(n, np.int32)
    d = np.empty(n, np.int32)
    v = np.empty(n, np.float64)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    k = _check(lib().pm_flux_entries(int(N), P(r, ctypes.c_int), P(c, ctypes.c_int),
                                     P(d, ctypes.c_int), P(v, ctypes.c_double), n))
    return r[:k], c[:k], d[:k], v[:k]


def pm_moment_grid(N, moment):
    return _check(lib().pm_moment_grid(int(N), int(moment)))


def pm_moment_slot(N, moment):
    return _check(lib().pm_moment_slot(int(N), int(moment)))


def pm_halo_plan(N, nx, ny, nz, parity, dirs=7, with_index=False):
    """Count of packed halo elements for a sweep of `parity` with the box
    split in the directions of `dirs` (bits x = 1, y = 2, z = 4); with_index:
    (count, moment array, cell array) in the packed order."""
    a = (int(N), int(nx), int(ny), int(nz), int(parity), int(dirs))
    n = _check(lib().pm_halo_plan(*a, None, None, 0))
    if not with_index:
        return n
    mom = np.empty(n, np.int64)
    cell = np.empty(n, np.int64)
    P = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))
    _check(lib().pm_halo_plan(*a, P(mom), P(cell), n))
    return n, mom, cell


def pm_halo_pack(parity, device_ptr, dirs=7):
    return _check(lib().pm_halo_pack(int(parity), int(dirs), ctypes.c_void_p(int(device_ptr))))


def pm_halo_unpack(parity, device_ptr, dirs=7):
    return _check(lib().pm_halo_unpack(int(parity), int(dirs), ctypes.c_void_p(int(device_ptr))))


def pm_device_bytes():
    return int(lib().pm_device_bytes())
