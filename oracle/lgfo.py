"""ctypes binding of the FP64 CPU oracle (oracle/lgfo.c).

TEST INFRASTRUCTURE ONLY (see lgfo.h).  Arrays are numpy complex128 in the
canonical layout: links (Lt, Lz, Ly, Lx, 4, 3, 3); per-site matrix fields
(Lt, Lz, Ly, Lx, 3, 3); dims = (Lx, Ly, Lz, Lt).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Opts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("theta_stop", C.c_double), ("max_iter", C.c_long),
                ("accel", C.c_int), ("store12", C.c_int), ("band_scale", C.POINTER(C.c_double)),
                ("expo", C.c_int)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liblgfo.so")
        if not os.path.exists(path):
            from .build import build
            build()
        L = C.CDLL(path)
        D, I4, P = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(Opts)
        L.lgfo_default_opts.argtypes = [P]
        L.lgfo_measure.argtypes = [I4, D, D, D, D]
        L.lgfo_fft4d.argtypes = [I4, D, C.c_int]
        L.lgfo_filter.argtypes = [P, I4, D, D]
        L.lgfo_gauge.argtypes = [I4, D, C.c_double, D]
        L.lgfo_gauge_exp.argtypes = [I4, D, C.c_double, D]
        L.lgfo_expm.argtypes = [D, C.c_long, D]
        L.lgfo_transform.argtypes = [I4, D, D, D]
        L.lgfo_step.argtypes = [P, I4, D, C.c_long, D, D, D]
        L.lgfo_fix.argtypes = [P, I4, D, C.POINTER(C.c_long), D, D, D]
        L.lgfo_plaquette.argtypes = [I4, D]
        L.lgfo_plaquette.restype = C.c_double
        L.lgfo_rebuild_row3.argtypes = [D, C.c_long]
        L.lgfo_unitarity.argtypes = [D, C.c_long, D, D]
        L.lgfo_band_index.argtypes = [I4, I4]
        L.lgfo_band_powers.argtypes = [I4, D, D, C.POINTER(C.c_long)]
        L.lgfo_threads.restype = C.c_int
        _LIB = L
    return _LIB


def _dims(dims):
    return (C.c_int * 4)(*[int(d) for d in dims])


def _dp(a):
    if a is None:
        return None
    assert a.flags.c_contiguous and a.dtype in (np.complex128, np.float64)
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _field_shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def opts(alpha=0.08, theta_stop=1e-15, max_iter=100000, accel=True, store12=False,
         band_scale=None, expo=False):
    o = Opts()
    lib().lgfo_default_opts(C.byref(o))
    o.alpha, o.theta_stop, o.max_iter = alpha, theta_stop, max_iter
    o.accel, o.store12, o.expo = int(bool(accel)), int(bool(store12)), int(bool(expo))
    if band_scale is not None:
        arr = np.ascontiguousarray(band_scale, dtype=np.float64)
        assert arr.shape == (16,)
        o._keep = arr
        o.band_scale = arr.ctypes.data_as(C.POINTER(C.c_double))
    return o


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments")
    return rc


def measure(dims, U):
    """(F, theta, Delta) of the links U."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    delta = np.empty(_field_shape(dims) + (3, 3), dtype=np.complex128)
    F, th = C.c_double(), C.c_double()
    _check(lib().lgfo_measure(_dims(dims), _dp(U), _dp(delta), C.byref(F), C.byref(th)), "measure")
    return F.value, th.value, delta


def fft4d(dims, field, sign=-1):
    f = np.array(field, dtype=np.complex128, order="C", copy=True)
    _check(lib().lgfo_fft4d(_dims(dims), _dp(f), int(sign)), "fft4d")
    return f


def filter_delta(dims, delta, o=None):
    o = o or opts()
    delta = np.ascontiguousarray(delta, dtype=np.complex128)
    out = np.empty_like(delta)
    _check(lib().lgfo_filter(C.byref(o), _dims(dims), _dp(delta), _dp(out)), "filter")
    return out


def gauge(dims, dtilde, alpha=0.08, expo=False):
    dtilde = np.ascontiguousarray(dtilde, dtype=np.complex128)
    g = np.empty_like(dtilde)
    fn = lib().lgfo_gauge_exp if expo else lib().lgfo_gauge
    _check(fn(_dims(dims), _dp(dtilde), float(alpha), _dp(g)), "gauge")
    return g


def expm(m):
    """exp of each 3x3 complex matrix in m (..., 3, 3), by the oracle's series."""
    m = np.ascontiguousarray(m, dtype=np.complex128)
    out = np.empty_like(m)
    _check(lib().lgfo_expm(_dp(m), m.size // 9, _dp(out)), "expm")
    return out


def transform(dims, U, g):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    g = np.ascontiguousarray(g, dtype=np.complex128)
    out = np.empty_like(U)
    _check(lib().lgfo_transform(_dims(dims), _dp(U), _dp(g), _dp(out)), "transform")
    return out


def step(dims, U, n, o=None, want_G=False):
    """n updates without a stop test: (U_n, trace_F[n+1], trace_theta[n+1], G or None)."""
    o = o or opts()
    U = np.array(U, dtype=np.complex128, order="C", copy=True)
    tf, tt = np.empty(n + 1), np.empty(n + 1)
    G = None
    if want_G:
        G = np.broadcast_to(np.eye(3, dtype=np.complex128), _field_shape(dims) + (3, 3)).copy()
    _check(lib().lgfo_step(C.byref(o), _dims(dims), _dp(U), int(n), _dp(tf), _dp(tt), _dp(G)), "step")
    return U, tf, tt, G


def fix(dims, U, o=None, want_G=False):
    """Iterate to theta < theta_stop: (U, iters, F, theta, converged, G or None)."""
    o = o or opts()
    U = np.array(U, dtype=np.complex128, order="C", copy=True)
    it, F, th = C.c_long(), C.c_double(), C.c_double()
    G = None
    if want_G:
        G = np.broadcast_to(np.eye(3, dtype=np.complex128), _field_shape(dims) + (3, 3)).copy()
    rc = _check(lib().lgfo_fix(C.byref(o), _dims(dims), _dp(U), C.byref(it), C.byref(F),
                               C.byref(th), _dp(G)), "fix")
    return U, it.value, F.value, th.value, rc == 0, G


def plaquette(dims, U):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    return lib().lgfo_plaquette(_dims(dims), _dp(U))


def rebuild_row3(m):
    m = np.array(m, dtype=np.complex128, order="C", copy=True)
    lib().lgfo_rebuild_row3(_dp(m), m.size // 9)
    return m


def unitarity(m):
    m = np.ascontiguousarray(m, dtype=np.complex128)
    a, b = C.c_double(), C.c_double()
    lib().lgfo_unitarity(_dp(m), m.size // 9, C.byref(a), C.byref(b))
    return a.value, b.value


def band_index(dims):
    b = np.empty(_field_shape(dims), dtype=np.int32)
    _check(lib().lgfo_band_index(_dims(dims), b.ctypes.data_as(C.POINTER(C.c_int))), "band_index")
    return b


def band_powers(dims, delta):
    delta = np.ascontiguousarray(delta, dtype=np.complex128)
    p = np.empty(16)
    c = (C.c_long * 16)()
    _check(lib().lgfo_band_powers(_dims(dims), _dp(delta), _dp(p), c), "band_powers")
    return p, np.array(c[:], dtype=np.int64)


def threads():
    return lib().lgfo_threads()
