"""Python binding of the C ABI in include/lgf.h (argument marshalling only).

Every step of the iteration runs in the HIP library liblgf.so built from
csrc/ for gfx950; this module only converts arguments.  If the library is
missing, loading fails with an error that says how to build it: there is no
fallback.

Arrays: links are complex128 (or float64 views) in the canonical layout
(Lt, Lz, Ly, Lx, 4, 3, 3); the gauge field G is (Lt, Lz, Ly, Lx, 3, 3);
dims are (Lx, Ly, Lz, Lt).  A torch tensor on the GPU is passed as a device
pointer (LGF_DEVICE); numpy arrays as host memory (LGF_HOST).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(_HERE, "liblgf.so")

OK = 0
E_INVALID_ARG, E_UNSUPPORTED_SHAPE, E_OUT_OF_MEMORY, E_DEVICE = -1, -2, -3, -4
E_NOT_UNITARY, E_NONFINITE, E_NOT_CONVERGED, E_STATE, E_MODEL = -5, -6, -7, -8, -9
HOST, DEVICE = 0, 1
FP64, FP32, MIXED = 0, 1, 2
STORE18, STORE12 = 18, 12
STEP_PLAIN, STEP_LEARNED = 0, 1
ACCEL_NONE, ACCEL_FOURIER = 0, 1
UPDATE_FIRST_ORDER, UPDATE_EXP = 0, 1


class Params(C.Structure):
    _fields_ = [("dims", C.c_int32 * 4), ("precision", C.c_int32), ("storage", C.c_int32),
                ("step", C.c_int32), ("accel", C.c_int32), ("update", C.c_int32),
                ("profile", C.c_int32), ("alpha", C.c_double), ("theta_stop", C.c_double),
                ("theta_switch", C.c_double), ("unit_tol", C.c_double), ("max_iter", C.c_int64),
                ("poll_every", C.c_int32), ("no_graph", C.c_int32), ("stream", C.c_void_p),
                ("autotune", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iter", C.c_int64), ("iter_fp32", C.c_int64), ("iter_fp64", C.c_int64),
                ("fallbacks", C.c_int64), ("F", C.c_double), ("theta", C.c_double),
                ("seconds", C.c_double), ("phase", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int32), ("seed", C.c_int32), ("lr", C.c_float),
                ("reserved", C.c_float)]


class LgfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_libs = {}


def load_library(path: str | None = None):
    """Load the C ABI library (default: the gfx950 build next to this file)."""
    path = os.path.abspath(path or os.environ.get("LGF_LIBRARY", DEFAULT_LIB))
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1206_0675_amd.build` "
                          "(hipcc --offload-arch=gfx950); there is no fallback implementation")
    L = C.CDLL(path)
    P, S, V, I32, I64 = C.POINTER(Params), C.POINTER(Stats), C.c_void_p, C.c_int32, C.c_int64
    ctx_p = C.POINTER(C.c_void_p)
    sig = {
        "lgf_default_params": ([P], I32),
        "lgf_validate_links": ([C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_double, C.POINTER(I64)], I32),
        "lgf_create": ([P, ctx_p], I32),
        "lgf_destroy": ([V], I32),
        "lgf_load_links": ([V, V, I32], I32),
        "lgf_store_links": ([V, V, I32], I32),
        "lgf_store_gauge": ([V, V, I32], I32),
        "lgf_load_gauge": ([V, V, I32], I32),
        "lgf_measure": ([V, S], I32),
        "lgf_step": ([V, I64, S], I32),
        "lgf_fix": ([V, S], I32),
        "lgf_profile_read": ([V, C.POINTER(I64), C.POINTER(C.c_double), I32, C.POINTER(I32)], I32),
        "lgf_profile_reset": ([V], I32),
        "lgf_kernel_name": ([I32], C.c_char_p),
        "lgf_device_bytes": ([V, C.POINTER(I64)], I32),
        "lgf_config": ([V, C.POINTER(I32), C.POINTER(I32)], I32),
        "lgf_strerror": ([I32], C.c_char_p),
        "lgf_last_error": ([V], C.c_char_p),
        "lgf_batch_create": ([P, I32, C.POINTER(C.c_int32 * 4), ctx_p], I32),
        "lgf_batch_destroy": ([V], I32),
        "lgf_batch_load": ([V, I32, V, I32], I32),
        "lgf_batch_fix": ([V, S], I32),
        "lgf_batch_store": ([V, I32, V, I32], I32),
        "lgf_batch_store_gauge": ([V, I32, V, I32], I32),
        "lgf_batch_config": ([V, C.POINTER(I32), C.POINTER(I32)], I32),
        "lgf_batch_last_error": ([V], C.c_char_p),
        "lgf_fix_batch": ([P, I32, C.POINTER(C.c_int32 * 4), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), S], I32),
        "lgf_fix_noalloc": ([P, V, V, S], I32),
        "lgf_noalloc_capacity": ([], C.c_size_t),
        "lgf_model_bytes": ([], C.c_size_t),
        "lgf_set_model": ([V, C.c_char_p, C.c_size_t], I32),
        "lgf_learned_factors": ([V, C.POINTER(C.c_double), C.POINTER(C.c_double)], I32),
        "lgf_linesearch_bands": ([V, C.POINTER(C.c_double), C.POINTER(C.c_double)], I32),
        "lgf_mlp_train": ([C.POINTER(C.c_float)] * 3 + [I64, C.POINTER(TrainParams), C.c_void_p,
                          C.POINTER(C.c_size_t), C.POINTER(C.c_float)], I32),
        "lgf_mlp_grad": ([C.c_char_p, C.c_size_t] + [C.POINTER(C.c_float)] * 3 + [I64, C.POINTER(C.c_float),
                         C.POINTER(C.c_double)], I32),
        "lgf_mlp_eval": ([C.c_char_p, C.c_size_t, C.POINTER(C.c_float), I64, C.POINTER(C.c_float)], I32),
        "lgf_wilson_create": ([C.POINTER(C.c_int32), C.c_double, C.c_uint64, ctx_p], I32),
        "lgf_wilson_destroy": ([V], I32),
        "lgf_wilson_cold": ([V], I32),
        "lgf_wilson_load": ([V, V, I32], I32),
        "lgf_wilson_sweep": ([V, I32], I32),
        "lgf_wilson_update": ([V, I64, I32], I32),
        "lgf_wilson_get_sweep": ([V, C.POINTER(C.c_uint64)], I32),
        "lgf_wilson_set_sweep": ([V, C.c_uint64], I32),
        "lgf_wilson_plaquette": ([V, C.POINTER(C.c_double)], I32),
        "lgf_wilson_store": ([V, V, I32], I32),
        "lgf_wilson_device_links": ([V], C.c_void_p),
        "lgf_wilson_skipped": ([V, C.POINTER(I64)], I32),
        "lgf_wilson_last_error": ([V], C.c_char_p),
        "lgf_fft_study": ([C.POINTER(C.c_int32), I32, V, V, I32, I32, C.POINTER(C.c_double)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes, fn.restype = args, res
    _libs[path] = L
    return L


def default_params(dims, lib=None, **kw) -> Params:
    L = lib or load_library()
    p = Params()
    L.lgf_default_params(C.byref(p))
    p.dims[:] = [int(d) for d in dims]
    for k, v in kw.items():
        if k == "stream":
            v = v if v is None or isinstance(v, int) else int(v)
        setattr(p, k, v)
    return p


def validate_links(dims, links, tol=1e-12, lib=None):
    """(status, first_bad) from the host-only check of canonical FP64 links."""
    L = lib or load_library()
    a = np.ascontiguousarray(links).view(np.float64)
    d = (C.c_int32 * 4)(*[int(x) for x in dims])
    bad = C.c_int64()
    rc = L.lgf_validate_links(d, a.ctypes.data_as(C.POINTER(C.c_double)), float(tol), C.byref(bad))
    return rc, bad.value


def _buffer(x):
    """(pointer, where, keepalive) for a numpy array or a torch tensor."""
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data, HOST, x
    if hasattr(x, "data_ptr") and hasattr(x, "is_cuda"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), (DEVICE if x.is_cuda else HOST), x
    raise TypeError("expected a numpy array or a torch tensor")


class Context:
    """One lattice configuration on the GPU (lgf_create ... lgf_destroy)."""

    def __init__(self, dims, lib=None, params: Params | None = None, **kw):
        self.lib = lib or load_library()
        self.dims = tuple(int(d) for d in dims)
        self.params = params if params is not None else default_params(self.dims, self.lib, **kw)
        h = C.c_void_p()
        rc = self.lib.lgf_create(C.byref(self.params), C.byref(h))
        if rc != OK:
            raise LgfError(rc, self.lib.lgf_last_error(None).decode())
        self.h = h

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.lgf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise LgfError(rc, self.lib.lgf_last_error(self.h).decode())
        return rc

    @property
    def shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx)

    # -- data --------------------------------------------------------------
    def load(self, links):
        ptr, where, _keep = _buffer(links)
        self._check(self.lib.lgf_load_links(self.h, C.c_void_p(ptr), where))

    def load_device(self, ptr: int):
        """Load links already in device memory (canonical layout) at address ptr."""
        self._check(self.lib.lgf_load_links(self.h, C.c_void_p(int(ptr)), DEVICE))

    def store(self, out=None):
        if out is None:
            out = np.empty(self.shape + (4, 3, 3), dtype=np.complex128)
        ptr, where, _keep = _buffer(out)
        self._check(self.lib.lgf_store_links(self.h, C.c_void_p(ptr), where))
        return out

    def store_gauge(self, out=None):
        if out is None:
            out = np.empty(self.shape + (3, 3), dtype=np.complex128)
        ptr, where, _keep = _buffer(out)
        self._check(self.lib.lgf_store_gauge(self.h, C.c_void_p(ptr), where))
        return out

    def load_gauge(self, G):
        ptr, where, _keep = _buffer(G)
        self._check(self.lib.lgf_load_gauge(self.h, C.c_void_p(ptr), where))

    # -- iteration ---------------------------------------------------------
    def measure(self) -> Stats:
        s = Stats()
        self._check(self.lib.lgf_measure(self.h, C.byref(s)))
        return s

    def step(self, n: int, trace: bool = False):
        """n updates; with trace, arrays (F[n+1], theta[n+1])."""
        if not trace:
            self._check(self.lib.lgf_step(self.h, int(n), None))
            return None
        tr = (Stats * (n + 1))()
        self._check(self.lib.lgf_step(self.h, int(n), tr))
        return np.array([t.F for t in tr]), np.array([t.theta for t in tr])

    def fix(self, raise_on_error=True) -> Stats:
        s = Stats()
        rc = self.lib.lgf_fix(self.h, C.byref(s))
        if raise_on_error:
            self._check(rc)
        return s

    # -- learned step ----------------------------------------------------------
    def set_model(self, blob: bytes):
        self._check(self.lib.lgf_set_model(self.h, blob, len(blob)))

    def learned_factors(self):
        x, s = (C.c_double * 16)(), (C.c_double * 16)()
        self._check(self.lib.lgf_learned_factors(self.h, x, s))
        return np.array(x[:]), np.array(s[:])

    def linesearch_bands(self):
        x, ls = (C.c_double * 16)(), (C.c_double * 16)()
        self._check(self.lib.lgf_linesearch_bands(self.h, x, ls))
        return np.array(x[:]), np.array(ls[:])

    # -- profiling -----------------------------------------------------------
    def profile(self):
        n = 32
        launches, ms, cnt = (C.c_int64 * n)(), (C.c_double * n)(), C.c_int32()
        self._check(self.lib.lgf_profile_read(self.h, launches, ms, n, C.byref(cnt)))
        out = {}
        for k in range(min(cnt.value, n)):
            if launches[k]:
                out[self.lib.lgf_kernel_name(k).decode()] = (int(launches[k]), float(ms[k]))
        return out

    def profile_reset(self):
        self._check(self.lib.lgf_profile_reset(self.h))

    def device_bytes(self):
        b = C.c_int64()
        self._check(self.lib.lgf_device_bytes(self.h, C.byref(b)))
        return b.value

    def config(self):
        """(threads per plane block, tile bytes) the context runs with."""
        a, b = C.c_int32(), C.c_int32()
        self._check(self.lib.lgf_config(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value


class Batch:
    """Many lattices of different shapes gauge-fixed together (lgf_batch_*)."""

    def __init__(self, dims_list, lib=None, params: Params | None = None, **kw):
        self.lib = lib or load_library()
        self.dims = [tuple(int(d) for d in dims) for dims in dims_list]
        self.n = len(self.dims)
        self.params = params if params is not None else default_params((0, 0, 0, 0), self.lib, **kw)
        arr = (C.c_int32 * 4 * self.n)(*[(C.c_int32 * 4)(*d) for d in self.dims])
        h = C.c_void_p()
        rc = self.lib.lgf_batch_create(C.byref(self.params), self.n, arr, C.byref(h))
        if rc != OK:
            raise LgfError(rc, self.lib.lgf_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lgf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise LgfError(rc, self.lib.lgf_batch_last_error(self.h).decode())
        return rc

    def _shape(self, i):
        lx, ly, lz, lt = self.dims[i]
        return (lt, lz, ly, lx)

    def load(self, i, links):
        ptr, where, _keep = _buffer(links)
        self._check(self.lib.lgf_batch_load(self.h, int(i), C.c_void_p(ptr), where))

    def fix(self, raise_on_error=True):
        out = (Stats * self.n)()
        rc = self.lib.lgf_batch_fix(self.h, out)
        if raise_on_error:
            self._check(rc)
        return list(out)

    def store(self, i, out=None):
        if out is None:
            out = np.empty(self._shape(i) + (4, 3, 3), dtype=np.complex128)
        ptr, where, _keep = _buffer(out)
        self._check(self.lib.lgf_batch_store(self.h, int(i), C.c_void_p(ptr), where))
        return out

    def store_gauge(self, i, out=None):
        if out is None:
            out = np.empty(self._shape(i) + (3, 3), dtype=np.complex128)
        ptr, where, _keep = _buffer(out)
        self._check(self.lib.lgf_batch_store_gauge(self.h, int(i), C.c_void_p(ptr), where))
        return out

    def config(self):
        a, b = C.c_int32(), C.c_int32()
        self._check(self.lib.lgf_batch_config(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value


def fix_batch(links_list, lib=None, **kw):
    """lgf_fix_batch on host arrays: returns (fixed links list, stats list, status)."""
    L = lib or load_library()
    n = len(links_list)
    dims = [(u.shape[3], u.shape[2], u.shape[1], u.shape[0]) for u in links_list]
    p = default_params((0, 0, 0, 0), L, **kw)
    ins = [np.ascontiguousarray(u, dtype=np.complex128) for u in links_list]
    outs = [np.empty_like(u) for u in ins]
    arr = (C.c_int32 * 4 * n)(*[(C.c_int32 * 4)(*d) for d in dims])
    pin = (C.c_void_p * n)(*[u.ctypes.data for u in ins])
    pout = (C.c_void_p * n)(*[u.ctypes.data for u in outs])
    st = (Stats * n)()
    rc = L.lgf_fix_batch(C.byref(p), n, arr, pin, pout, st)
    return outs, list(st), rc


def fix_noalloc(links_in, links_out, lib=None, **kw):
    """lgf_fix_noalloc: gauge-fix device-resident canonical links (torch
    tensors on the GPU) with no device allocation by the library.  dims come
    from the tensor shape (Lt, Lz, Ly, Lx, 4, 3, 3); returns (stats, status)."""
    L = lib or load_library()
    for t in (links_in, links_out):
        if not (hasattr(t, "is_cuda") and t.is_cuda and t.is_contiguous()):
            raise ValueError("lgf_fix_noalloc takes contiguous device tensors")
    sh = tuple(links_in.shape)
    p = default_params((sh[3], sh[2], sh[1], sh[0]), L, **kw)
    st = Stats()
    rc = L.lgf_fix_noalloc(C.byref(p), C.c_void_p(links_in.data_ptr()), C.c_void_p(links_out.data_ptr()),
                           C.byref(st))
    return st, rc


def _f32(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def mlp_train(X, Y, M, steps=2000, batch=256, seed=1, lr=1e-3, lib=None):
    """Train the learned-step network on the GPU: (model blob, loss per step)."""
    L = lib or load_library()
    X, px = _f32(X)
    Y, py = _f32(Y)
    M, pm = _f32(M)
    n = X.shape[0]
    tp = TrainParams(steps=int(steps), batch=int(batch), seed=int(seed), lr=float(lr))
    cap = C.c_size_t(L.lgf_model_bytes())
    blob = C.create_string_buffer(cap.value)
    trace = np.zeros(max(int(steps), 1), dtype=np.float32)
    rc = L.lgf_mlp_train(px, py, pm, n, C.byref(tp), blob, C.byref(cap), trace.ctypes.data_as(C.POINTER(C.c_float)))
    if rc != OK:
        raise LgfError(rc, L.lgf_last_error(None).decode())
    return blob.raw[:cap.value], trace[:int(steps)]


def mlp_grad(blob, X, Y, M, lib=None):
    """(loss, gradient[6288]) of a model on samples, by the training kernels."""
    L = lib or load_library()
    X, px = _f32(X)
    Y, py = _f32(Y)
    M, pm = _f32(M)
    g = np.zeros(6288, dtype=np.float32)
    loss = C.c_double()
    rc = L.lgf_mlp_grad(blob, len(blob), px, py, pm, X.shape[0], g.ctypes.data_as(C.POINTER(C.c_float)),
                        C.byref(loss))
    if rc != OK:
        raise LgfError(rc, L.lgf_last_error(None).decode())
    return loss.value, g


def mlp_eval(blob, X, lib=None):
    L = lib or load_library()
    X, px = _f32(X)
    Y = np.zeros_like(X)
    rc = L.lgf_mlp_eval(blob, len(blob), px, X.shape[0], Y.ctypes.data_as(C.POINTER(C.c_float)))
    if rc != OK:
        raise LgfError(rc, L.lgf_last_error(None).decode())
    return Y


# ---------------------------------------------------------------------------
# Wilson-action configuration generator (include/lgf_wilson.h)
# ---------------------------------------------------------------------------
HEATBATH, OVERRELAX = 0, 1


class WilsonGenerator:
    """Heatbath + overrelaxation generator of Wilson-action SU(3) links on the
    GPU (lgf_wilson_create ... lgf_wilson_destroy); links start cold."""

    def __init__(self, dims, beta: float, seed: int, lib=None):
        self.lib = lib or load_library()
        self.dims = tuple(int(d) for d in dims)
        h = C.c_void_p()
        d = (C.c_int32 * 4)(*self.dims)
        rc = self.lib.lgf_wilson_create(d, float(beta), int(seed), C.byref(h))
        if rc != OK:
            raise LgfError(rc, self.lib.lgf_wilson_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lgf_wilson_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise LgfError(rc, self.lib.lgf_wilson_last_error(self.h).decode())
        return rc

    @property
    def shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx, 4, 3, 3)

    def cold(self):
        self._check(self.lib.lgf_wilson_cold(self.h))

    def load(self, links):
        ptr, where, _keep = _buffer(links)
        self._check(self.lib.lgf_wilson_load(self.h, C.c_void_p(ptr), where))

    def sweep(self, kind: int = HEATBATH):
        self._check(self.lib.lgf_wilson_sweep(self.h, int(kind)))

    def update(self, n_update: int, n_or: int = 4):
        self._check(self.lib.lgf_wilson_update(self.h, int(n_update), int(n_or)))

    @property
    def sweep_index(self) -> int:
        n = C.c_uint64()
        self._check(self.lib.lgf_wilson_get_sweep(self.h, C.byref(n)))
        return n.value

    @sweep_index.setter
    def sweep_index(self, n: int):
        self._check(self.lib.lgf_wilson_set_sweep(self.h, int(n)))

    def plaquette(self) -> float:
        p = C.c_double()
        self._check(self.lib.lgf_wilson_plaquette(self.h, C.byref(p)))
        return p.value

    def store(self, out=None):
        if out is None:
            out = np.empty(self.shape, dtype=np.complex128)
        ptr, where, _keep = _buffer(out)
        self._check(self.lib.lgf_wilson_store(self.h, C.c_void_p(ptr), where))
        return out

    @property
    def device_links(self) -> int:
        """Device address of the links (canonical layout), for Context.load_device;
        holds the links of the last sweep, cold start or load."""
        p = self.lib.lgf_wilson_device_links(self.h)
        if not p:
            raise LgfError(E_DEVICE, self.lib.lgf_wilson_last_error(self.h).decode())
        return p

    def skipped(self) -> int:
        n = C.c_int64()
        self._check(self.lib.lgf_wilson_skipped(self.h, C.byref(n)))
        return n.value


# ---------------------------------------------------------------------------
# FFT decomposition study (include/lgf_study.h)
# ---------------------------------------------------------------------------
FFT_1DX4, FFT_2D1D1D, FFT_2D2D, FFT_2D1D1D_MFMA = 0, 1, 2, 3


def fft_study(dims, variant: int, fields, out=None, reps: int = 0, lib=None):
    """(out, ms per filter): F^-1 (p2max/p^2) F / V of four complex fields in
    the plain layout (4, Lt, Lz, Ly, Lx), by the given decomposition."""
    L = lib or load_library()
    if out is None:
        out = np.empty_like(fields) if isinstance(fields, np.ndarray) else fields.new_empty(fields.shape)
    pin, win, _k1 = _buffer(fields)
    pout, wout, _k2 = _buffer(out)
    if win != wout:
        raise ValueError("fields and out must both be host or both be device memory")
    ms = C.c_double()
    d = (C.c_int32 * 4)(*[int(x) for x in dims])
    rc = L.lgf_fft_study(d, int(variant), C.c_void_p(pin), C.c_void_p(pout), win, int(reps), C.byref(ms))
    if rc != OK:
        raise LgfError(rc, L.lgf_last_error(None).decode())
    return out, ms.value
