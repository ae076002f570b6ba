"""Seeded synthetic SU(3) gauge fields for Landau gauge fixing.

This module only *draws inputs*: it holds none of the gauge-fixing method's
arithmetic (no gradient field, no Fourier acceleration, no functional, no
reunitarisation).  Both the FP64 oracle and the GPU library are fed from here,
so the two never share any code path beyond the input arrays.

Layout ("canonical"): a complex128 array of shape (Lt, Lz, Ly, Lx, 4, 3, 3),
i.e. x fastest, then the direction mu = 0..3 (x, y, z, t), then the 3x3 matrix
in row-major order.  Viewed as float64 it is 72 doubles per site.  `dims` is
always given as (Lx, Ly, Lz, Lt).

Workload (the paper measures on Wilson-action ensembles that are not
available; these fields stand in for them, see the paper's Section 4):

    U_mu(x) = g(x) exp(i eps H_mu(x)) g^dagger(x + mu)

with g Haar-random in SU(3), H = sum_a h_a lambda_a / 2 (Gell-Mann matrices,
h_a iid standard normal), and eps chosen so the mean plaquette is about 0.6.
The gauge rotation g makes the field far from Landau gauge while keeping the
gauge-invariant content of exp(i eps H).

Random numbers: a counter-based SplitMix64 stream.  Output i of the stream
with key k is mix64(k + (i + 1) * 0x9E3779B97F4A7C15), where mix64 is the
SplitMix64 finaliser (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).  Uniforms take the top 53 bits; normals use the
cosine branch of Box-Muller on consecutive uniform pairs.  Haar matrices use
the QR method with the phase fix of Mezzadri ("How to generate random
matrices from the classical compact groups", Notices AMS 54, 2007).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "EPS_PLAQ_06",
    "GELL_MANN",
    "normals",
    "haar_su3",
    "algebra_exp",
    "random_links",
    "pure_gauge",
    "small_field",
    "identity_links",
    "volume",
    "calibrate_eps",
]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream kinds (the low byte of the stream key).
KIND_ALGEBRA = 1   # 8 normals per (site, mu): the h_a of H_mu(x)
KIND_HAAR = 2      # 18 normals per site: the Ginibre matrix behind g(x)
KIND_CALIB = 3     # plaquette calibration sample

# eps such that the mean plaquette of the generated fields is 0.600.
# Reproduced by calibrate_eps(0.6) (bisection on a 2^20-plaquette sample).
EPS_PLAQ_06 = 0.4324951171875


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, kind: int) -> np.uint64:
    z = np.array([(int(seed) << 8 | int(kind)) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(z + _GAMMA)[0]


def _uniforms(key: np.uint64, start: int, count: int) -> np.ndarray:
    """Uniforms in [0, 1): outputs start .. start+count-1 of stream `key`."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix64(key + i * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normals(seed: int, kind: int, start: int, count: int) -> np.ndarray:
    """Standard normals number start .. start+count-1 of stream (seed, kind).

    Normal k uses uniforms 2k and 2k+1: sqrt(-2 ln(1 - u0)) cos(2 pi u1).
    """
    u = _uniforms(_key(seed, kind), 2 * start, 2 * count).reshape(count, 2)
    return np.sqrt(-2.0 * np.log1p(-u[:, 0])) * np.cos(2.0 * np.pi * u[:, 1])


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return lam


GELL_MANN = _gell_mann()


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def _check_dims(dims):
    if len(dims) != 4 or any(int(d) < 1 for d in dims):
        raise ValueError(f"dims must be four positive extents, got {dims!r}")


def haar_su3(seed: int, n: int, start: int = 0, kind: int = KIND_HAAR) -> np.ndarray:
    """n Haar-random SU(3) matrices (indices start .. start+n-1 of the stream)."""
    z = normals(seed, kind, 18 * start, 18 * n).reshape(n, 3, 3, 2)
    z = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]          # Mezzadri phase fix: Haar on U(3)
    det = np.linalg.det(q)
    return q * np.exp(-1j * np.angle(det) / 3.0)[:, None, None]   # into SU(3)


def algebra_exp(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for H = sum_a h_a lambda_a / 2; h has shape (n, 8)."""
    H = np.einsum("na,aij->nij", h, GELL_MANN) * 0.5
    w, v = np.linalg.eigh(H)
    return (v * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))


def _shift_minus(a: np.ndarray, mu: int) -> np.ndarray:
    """b[x] = a[x + mu] on a (Lt, Lz, Ly, Lx, ...) periodic array."""
    axis = 3 - mu
    return np.roll(a, -1, axis=axis)


def _algebra_links(dims, seed: int, eps: float) -> np.ndarray:
    lx, ly, lz, lt = dims
    V = volume(dims)
    out = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    slab = lx * ly * lz
    for t in range(lt):                       # one time slice at a time: bounded memory
        h = normals(seed, KIND_ALGEBRA, t * slab * 32, slab * 32).reshape(slab * 4, 8)
        out[t] = algebra_exp(h, eps).reshape(lz, ly, lx, 4, 3, 3)
    assert out.size == V * 36
    return out


def _gauge_field(dims, seed: int) -> np.ndarray:
    lx, ly, lz, lt = dims
    slab = lx * ly * lz
    g = np.empty((lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    for t in range(lt):
        g[t] = haar_su3(seed, slab, start=t * slab).reshape(lz, ly, lx, 3, 3)
    return g


def _rotate(links: np.ndarray, g: np.ndarray) -> np.ndarray:
    out = np.empty_like(links)
    for mu in range(4):
        gp = np.conj(np.swapaxes(_shift_minus(g, mu), -1, -2))
        out[..., mu, :, :] = g @ links[..., mu, :, :] @ gp
    return out


def _rotated_slice(args) -> np.ndarray:
    """Time slice t of g exp(i eps H) g^dag(x + mu): the same arithmetic as
    _rotate on the whole field, so the result is bitwise the same."""
    dims, seed, eps, t = args
    lx, ly, lz, lt = dims
    slab = lx * ly * lz
    h = normals(seed, KIND_ALGEBRA, t * slab * 32, slab * 32).reshape(slab * 4, 8)
    links = algebra_exp(h, eps).reshape(lz, ly, lx, 4, 3, 3)
    g = haar_su3(seed, slab, start=t * slab).reshape(lz, ly, lx, 3, 3)
    t1 = (t + 1) % lt
    g_next = haar_su3(seed, slab, start=t1 * slab).reshape(lz, ly, lx, 3, 3)
    out = np.empty_like(links)
    for mu in range(4):
        gn = g_next if mu == 3 else np.roll(g, -1, axis=2 - mu)
        out[..., mu, :, :] = g @ links[..., mu, :, :] @ np.conj(np.swapaxes(gn, -1, -2))
    return out


def random_links(dims, seed: int, eps: float = EPS_PLAQ_06, rotate: bool = True, workers: int = 1) -> np.ndarray:
    """U_mu(x) = g(x) exp(i eps H_mu(x)) g^dagger(x + mu)  (canonical layout).

    workers > 1 generates one time slice per task in that many worker
    processes (fresh interpreters, numpy only); each slice depends only on the
    counter streams, so the result is bitwise the same for any worker count.
    Only call it that way from a process that has not touched a GPU: the
    workers are started by fork and exec."""
    _check_dims(dims)
    dims = tuple(int(d) for d in dims)
    if not rotate:
        return _algebra_links(dims, seed, eps)
    if workers <= 1 or volume(dims) < (1 << 16):
        return _rotate(_algebra_links(dims, seed, eps), _gauge_field(dims, seed))
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    lx, ly, lz, lt = dims
    out = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for t, sl in enumerate(ex.map(_rotated_slice, [(dims, seed, eps, t) for t in range(lt)])):
            out[t] = sl
    return out


def small_field(dims, seed: int, eps: float = 1e-5) -> np.ndarray:
    """exp(i eps H_mu(x)) with no gauge rotation: the linear regime."""
    return random_links(dims, seed, eps, rotate=False)


def pure_gauge(dims, seed: int) -> np.ndarray:
    """U_mu(x) = h(x) h^dagger(x + mu): a point on the gauge orbit of U = 1."""
    _check_dims(dims)
    dims = tuple(int(d) for d in dims)
    lx, ly, lz, lt = dims
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), (lt, lz, ly, lx, 4, 3, 3)).copy()
    return _rotate(eye, _gauge_field(dims, seed))


def identity_links(dims) -> np.ndarray:
    _check_dims(dims)
    lx, ly, lz, lt = (int(d) for d in dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (lt, lz, ly, lx, 4, 3, 3)).copy()


def _plaquette_sample(eps: float, n: int, seed: int = 7) -> float:
    """Mean Re Tr(U1 U2 U3^dag U4^dag)/3 over n plaquettes of iid links.

    The generated fields have iid links before the gauge rotation, and the
    plaquette is gauge invariant, so this is their expected mean plaquette.
    """
    h = normals(seed, KIND_CALIB, 0, n * 32).reshape(n * 4, 8)
    u = algebra_exp(h, eps).reshape(n, 4, 3, 3)
    d = lambda m: np.conj(np.swapaxes(m, -1, -2))
    p = u[:, 0] @ u[:, 1] @ d(u[:, 2]) @ d(u[:, 3])
    return float(np.mean(np.real(np.trace(p, axis1=1, axis2=2))) / 3.0)


def calibrate_eps(target: float = 0.6, n: int = 1 << 20, lo: float = 0.0, hi: float = 1.0,
                  steps: int = 12) -> float:
    """Bisect eps so the expected mean plaquette equals `target`."""
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if _plaquette_sample(mid, n) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
