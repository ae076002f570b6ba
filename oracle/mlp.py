"""FP64 reference of the learned spectral step (TEST INFRASTRUCTURE ONLY).

The learned step replaces the fixed factor (alpha/2) p2max/p^2 of eq. gx by
s_b (alpha/2) p2max/p^2, with one factor s_b per band of |p^2| (16 bands,
log-spaced between the smallest nonzero p^2 of the lattice and p2max, the
zero mode excluded).  A small network maps the band powers of Delta to the
factors:

    P_b   = mean over the modes p of band b of sum_c |Dhat_c(p)|^2
            (c over the four complex fields holding Delta's 8 real
            components; unnormalised forward FFT)
    x_b   = log10(max(P_b / V, 1e-300)) / 8      (0 for an empty band)
    h1    = relu(x W1 + b1)         W1: 16 x 64
    h2    = relu(h1 W2 + b2)        W2: 64 x 64
    y     = h2 W3 + b3              W3: 64 x 16
    s_b   = exp(clip(y_b, -2.3, 2.3))

Weights are stored in bfloat16 (round to nearest even from float32) and
biases in float32; this reference evaluates the network in float64 on those
exact values.  The factors an update applies come from the network on the band powers
of the previous update's spectrum (s = 1 for the first update after a load):
the spectrum of the current links is only known once the update's own
(z, t) pass has run, so the factors lag it by one update.  An update with
factors s is accepted if it increases F or lowers theta; otherwise the plain
update (s = 1) is taken.  (Near convergence the gain in F per update falls
below the rounding of F while theta still resolves it, so a test on F alone
would reject good candidates there.)

Training targets: the one factor s, common to all bands, that minimises theta
after one update (theta is what the stop test reads, and it stays resolvable
down to 1e-15, where the gain in F is lost in rounding), found by
golden-section search on ln s in [-2.3, 2.3] and kept only if it beats the
plain step; it is the target of every band that holds modes.  (Choosing each
band's factor greedily starves the slow low-momentum bands and lengthens the
run.)  The loss is the masked mean squared error over the bands that hold
modes.
"""
from __future__ import annotations

import numpy as np

from . import lgfo

NB, H1, H2 = 16, 64, 64
CLIP = 2.3
SHAPES = [("W1", (NB, H1)), ("b1", (H1,)), ("W2", (H1, H2)), ("b2", (H2,)), ("W3", (H2, NB)), ("b3", (NB,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
MAGIC = 0x4C47464D   # "LGFM"


# --------------------------------------------------------------------------
# bfloat16
# --------------------------------------------------------------------------
def to_bf16_bits(a) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest even (finite inputs)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# model blob: int32 header {magic, version, 16, 64, 64, 16, 0, 0},
# bf16 W1, W2, W3 (row-major [in][out]), float32 b1, b2, b3
# --------------------------------------------------------------------------
def blob_from_params(p: dict) -> bytes:
    head = np.array([MAGIC, 1, NB, H1, H2, NB, 0, 0], dtype=np.int32).tobytes()
    w = b"".join(to_bf16_bits(p[k]).tobytes() for k in ("W1", "W2", "W3"))
    b = b"".join(np.asarray(p[k], dtype=np.float32).tobytes() for k in ("b1", "b2", "b3"))
    return head + w + b


def params_from_blob(blob: bytes) -> dict:
    head = np.frombuffer(blob[:32], dtype=np.int32)
    if head[0] != MAGIC or head[1] != 1 or tuple(head[2:6]) != (NB, H1, H2, NB):
        raise ValueError("not a learned-step model blob")
    off = 32
    out = {}
    for k, shp in (("W1", (NB, H1)), ("W2", (H1, H2)), ("W3", (H2, NB))):
        n = int(np.prod(shp))
        out[k] = from_bf16_bits(np.frombuffer(blob[off:off + 2 * n], dtype=np.uint16)).reshape(shp)
        off += 2 * n
    for k, n in (("b1", H1), ("b2", H2), ("b3", NB)):
        out[k] = np.frombuffer(blob[off:off + 4 * n], dtype=np.float32).astype(np.float64)
        off += 4 * n
    if off != len(blob):
        raise ValueError("model blob has the wrong size")
    return out


def flat(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k, _ in SHAPES])


def unflat(v: np.ndarray) -> dict:
    out, off = {}, 0
    for k, shp in SHAPES:
        n = int(np.prod(shp))
        out[k] = v[off:off + n].reshape(shp)
        off += n
    return out


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------
def forward(p: dict, x: np.ndarray):
    """y for inputs x (n, 16); also the activations for backward."""
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(p: dict, x, t, m):
    """Masked mean squared error sum(m (y - t)^2) / sum(m) and its gradient."""
    y, (x, z1, h1, z2, h2) = forward(p, x)
    msum = float(np.sum(m))
    r = (y - t) * m
    loss = float(np.sum(r * (y - t)) / msum)
    d3 = 2.0 * r / msum
    g = {"W3": h2.T @ d3, "b3": d3.sum(0)}
    d2 = (d3 @ p["W3"].T) * (z2 > 0)
    g["W2"], g["b2"] = h1.T @ d2, d2.sum(0)
    d1 = (d2 @ p["W2"].T) * (z1 > 0)
    g["W1"], g["b1"] = x.T @ d1, d1.sum(0)
    return loss, g


def features(power16, count16, V):
    x = np.zeros(NB)
    for b in range(NB):
        if count16[b] > 0:
            x[b] = np.log10(max(power16[b] / V, 1e-300)) / 8.0
    return x


def factors(p: dict, x):
    y, _ = forward(p, np.asarray(x, dtype=np.float64)[None, :])
    return np.exp(np.clip(y[0], -CLIP, CLIP))


# --------------------------------------------------------------------------
# the learned update (FP64), following the plain step of Algorithm 1
# --------------------------------------------------------------------------
def update_with(dims, U, s, alpha=0.08):
    """One update with per-band factors s (s = None: the plain update)."""
    _, _, delta = lgfo.measure(dims, U)
    o = lgfo.opts(alpha=alpha, band_scale=None if s is None else np.asarray(s, dtype=np.float64))
    g = lgfo.gauge(dims, lgfo.filter_delta(dims, delta, o), alpha)
    return lgfo.transform(dims, U, g)


def learned_step(dims, U, p: dict, s, alpha=0.08):
    """One learned update with the factors s it was handed (s = None: the
    plain factors).  Returns (U', accepted, s_next, x): the candidate from s
    is kept iff it raises F or lowers theta, else the plain update is taken;
    x are the
    features of the band powers of U's spectrum and s_next the network's
    factors for them, which the next update uses (the factors lag the
    spectrum by one update)."""
    V = int(np.prod(dims))
    F0, th0, delta = lgfo.measure(dims, U)
    P, cnt = lgfo.band_powers(dims, delta)
    x = features(P, cnt, V)
    s_next = factors(p, x)
    U1 = update_with(dims, U, s, alpha)
    F1, th1, _ = lgfo.measure(dims, U1)
    if F1 > F0 or th1 < th0:
        return U1, True, s_next, x
    return update_with(dims, U, None, alpha), False, s_next, x


def learned_run(dims, U, p: dict, n=None, theta_stop=1e-15, max_iter=100000, alpha=0.08):
    """n learned updates from freshly loaded links (s = 1 for the first), or,
    with n = None, updates until theta < theta_stop.  Returns (U, iterations,
    fallbacks, F, theta)."""
    s, it, fb = None, 0, 0
    while True:
        F, th, _ = lgfo.measure(dims, U)
        if (n is not None and it >= n) or (n is None and (th < theta_stop or it >= max_iter)):
            return U, it, fb, F, th
        U, ok, s, _ = learned_step(dims, U, p, s, alpha)
        fb += 0 if ok else 1
        it += 1


def linesearch(dims, U, alpha=0.08, iters=20):
    """Log factors minimising theta after one update with one factor s for all
    bands: golden-section search on ln s in [-2.3, 2.3]; s = 1 unless the
    search beat the plain step.  Returns (features, log s per band: ln s for
    every band that holds modes and 0 for empty ones, best theta)."""
    V = int(np.prod(dims))
    _, _, delta = lgfo.measure(dims, U)
    P, cnt = lgfo.band_powers(dims, delta)
    x = features(P, cnt, V)

    def f(u):
        return lgfo.measure(dims, update_with(dims, U, np.full(NB, np.exp(u)), alpha))[1]

    best = lgfo.measure(dims, update_with(dims, U, np.ones(NB), alpha))[1]
    g = 0.5 * (np.sqrt(5.0) - 1.0)
    lo, hi = -CLIP, CLIP
    u1, u2 = hi - g * (hi - lo), lo + g * (hi - lo)
    f1, f2 = f(u1), f(u2)
    for _ in range(iters):
        if f1 < f2:
            hi, u2, f2 = u2, u1, f1
            u1 = hi - g * (hi - lo)
            f1 = f(u1)
        else:
            lo, u1, f1 = u1, u2, f2
            u2 = lo + g * (hi - lo)
            f2 = f(u2)
    u, fu = (u1, f1) if f1 < f2 else (u2, f2)
    ls = np.zeros(NB)
    if fu < best:
        best = fu
        ls[np.asarray(cnt) > 0] = u
    return x, ls, best
