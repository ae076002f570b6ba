"""ctypes binding of the Wilson-action generator reference (oracle/wilson.c).

TEST INFRASTRUCTURE ONLY (see wilson.h).  Links are numpy complex128 in the
canonical layout (Lt, Lz, Ly, Lx, 4, 3, 3); dims = (Lx, Ly, Lz, Lt), every
extent even.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lgfo

MAX_ATTEMPTS = 1024
HEATBATH, OVERRELAX = 0, 1

_BOUND = False


def lib():
    global _BOUND
    L = lgfo.lib()
    if not _BOUND:
        D, I4, U64 = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_uint64
        L.wilsono_philox4x64.argtypes = [C.POINTER(U64), C.POINTER(U64), C.POINTER(U64)]
        L.wilsono_philox4x64.restype = None
        L.wilsono_x0_sample.argtypes = [C.c_double, U64, C.c_long, D, C.POINTER(C.c_long)]
        L.wilsono_staple.argtypes = [I4, D, C.c_long, C.c_int, D]
        L.wilsono_link_action_sum.argtypes = [I4, D]
        L.wilsono_link_action_sum.restype = C.c_double
        L.wilsono_link_update.argtypes = [I4, D, C.c_long, C.c_int, C.c_double, U64, U64, C.c_int,
                                          C.POINTER(C.c_long)]
        L.wilsono_sweep.argtypes = [I4, D, C.c_double, U64, U64, C.c_int, C.POINTER(C.c_long)]
        L.wilsono_cold.argtypes = [I4, D]
        L.wilsono_generate.argtypes = [I4, D, C.c_double, U64, U64, C.c_long, C.c_int, C.POINTER(C.c_long)]
        _BOUND = True
    return L


def _dims(dims):
    return (C.c_int * 4)(*[int(d) for d in dims])


def _dp(a):
    assert a.flags.c_contiguous and a.dtype == np.complex128
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments")
    return rc


def philox4x64(counter, key):
    """The four 64-bit outputs of Philox4x64-10 for one counter and key."""
    c = (C.c_uint64 * 4)(*[int(v) for v in counter])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    lib().wilsono_philox4x64(c, k, o)
    return [int(v) for v in o]


def x0_sample(c, seed, n):
    """(draws, failed): n draws of the x0 sampler for sqrt(1-x^2) exp(c x)."""
    out = np.empty(int(n))
    f = C.c_long()
    _check(lib().wilsono_x0_sample(float(c), int(seed), int(n), out.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(f)), "x0_sample")
    return out, f.value


def staple(dims, U, site, mu):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    _check(lib().wilsono_staple(_dims(dims), _dp(U), int(site), int(mu), _dp(out)), "staple")
    return out


def link_action_sum(dims, U):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    return lib().wilsono_link_action_sum(_dims(dims), _dp(U))


def link_update(dims, U, site, mu, beta, seed, sweep, kind):
    """(U', skipped) after one heatbath (kind 0) or overrelaxation (1) link update."""
    U = np.array(U, dtype=np.complex128, order="C", copy=True)
    sk = C.c_long()
    _check(lib().wilsono_link_update(_dims(dims), _dp(U), int(site), int(mu), float(beta), int(seed), int(sweep),
                                     int(kind), C.byref(sk)), "link_update")
    return U, sk.value


def sweep(dims, U, beta, seed, n, kind):
    """(U', skipped) after one sweep: heatbath numbered n (kind 0) or overrelaxation (1)."""
    U = np.array(U, dtype=np.complex128, order="C", copy=True)
    sk = C.c_long()
    _check(lib().wilsono_sweep(_dims(dims), _dp(U), float(beta), int(seed), int(n), int(kind), C.byref(sk)),
           "sweep")
    return U, sk.value


def cold(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    U = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    _check(lib().wilsono_cold(_dims(dims), _dp(U)), "cold")
    return U


def generate(dims, U, beta, seed, first_sweep, n_update, n_or):
    """(U', skipped): n_update times one heatbath sweep then n_or overrelaxation sweeps."""
    U = np.array(U, dtype=np.complex128, order="C", copy=True)
    sk = C.c_long()
    _check(lib().wilsono_generate(_dims(dims), _dp(U), float(beta), int(seed), int(first_sweep), int(n_update),
                                  int(n_or), C.byref(sk)), "generate")
    return U, sk.value
