"""Pins of the FP64 reference of the learned spectral step (oracle/mlp.py)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import mlp


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = {k: rng.normal(scale=scale, size=s) for k, s in mlp.SHAPES}
    return mlp.params_from_blob(mlp.blob_from_params(p))     # bf16 weights, f32 biases


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0, 1e-30]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(mlp.to_bf16_bits(a), ref)


def test_blob_roundtrip():
    p = random_params(2)
    q = mlp.params_from_blob(mlp.blob_from_params(p))
    for k, _ in mlp.SHAPES:
        assert np.array_equal(p[k], q[k])
    assert len(mlp.blob_from_params(p)) == 32 + 2 * 6144 + 4 * 144 and mlp.NPARAM == 6288


def test_gradient_matches_finite_differences():
    p = random_params(3)
    rng = np.random.default_rng(4)
    x, t = rng.normal(size=(20, 16)), rng.normal(size=(20, 16))
    m = (rng.random((20, 16)) > 0.3).astype(float)
    loss, g = mlp.loss_and_grad(p, x, t, m)
    v, gv = mlp.flat(p), mlp.flat(g)
    for i in rng.choice(mlp.NPARAM, 60, replace=False):
        h = 1e-6
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fd = (mlp.loss_and_grad(mlp.unflat(vp), x, t, m)[0] - mlp.loss_and_grad(mlp.unflat(vm), x, t, m)[0]) / (2 * h)
        assert abs(fd - gv[i]) <= 1e-6 * max(1.0, abs(gv[i]))


def test_band_powers_parseval_and_counts(oracle_lib):
    dims = (8, 8, 4, 8)
    V = synth.volume(dims)
    _, _, d = oracle.measure(dims, synth.random_links(dims, 3))
    P, cnt = oracle.band_powers(dims, d)
    fields = np.stack([d[..., 0, 1], d[..., 0, 2], d[..., 1, 2], d[..., 0, 0].imag + 1j * d[..., 1, 1].imag])
    total = V * np.sum(np.abs(fields) ** 2)          # Parseval; the p = 0 mode carries sum_x Delta = 0
    assert abs(np.sum(P * cnt) - total) <= 1e-10 * total
    assert cnt.sum() == V - 1
    band = oracle.band_index(dims)
    assert band.ravel()[0] == -1
    p2 = sum(4 * np.sin(np.pi * c / L) ** 2 for c, L in zip(np.meshgrid(*[np.arange(L) for L in dims[::-1]],
                                                                          indexing="ij")[::-1], dims))
    assert np.all(band[p2 == p2.max()] == 15)
    assert np.all(band[np.isclose(p2, p2[p2 > 0].min())] == 0)


def test_zero_network_is_the_plain_step(oracle_lib):
    """A network that outputs 0 gives s = 1 everywhere: every learned update
    is the plain update, bit for bit."""
    dims = (4, 4, 8, 4)
    U = synth.random_links(dims, 5)
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    U1, acc, s, x = mlp.learned_step(dims, U, p, None)
    assert np.all(s == 1.0)
    Up, _, _, _ = oracle.step(dims, U, 1)
    assert np.array_equal(U1, Up)
    U3, it, fb, _, _ = mlp.learned_run(dims, U, p, n=3)
    assert it == 3 and np.array_equal(U3, oracle.step(dims, U, 3)[0])


def test_factor_too_large_falls_back(oracle_lib):
    # linear regime: the update multiplies every mode of Delta by 1 - 0.08 * 16 * s;
    # s = e^2.3 ~ 10 gives |1 - 12.8| > 1, so F drops and theta grows, and the
    # plain step is taken
    dims = (4, 4, 8, 4)
    U = synth.small_field(dims, 5, eps=1e-3)
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["b3"] = np.full(16, 2.3)
    U1, acc, s, x = mlp.learned_step(dims, U, p, np.full(16, np.exp(2.3)))
    assert not acc
    assert np.array_equal(U1, oracle.step(dims, U, 1)[0])
    assert np.allclose(s, np.exp(2.3))


def test_factors_lag_the_spectrum_by_one_update(oracle_lib):
    """The first update after a load applies s = 1; update n + 1 applies the
    network's factors for the band powers of update n's spectrum."""
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 11)
    rng = np.random.default_rng(12)
    p = {k: rng.normal(scale=0.2, size=sh) for k, sh in mlp.SHAPES}
    V = synth.volume(dims)
    U1, _, s1, x0 = mlp.learned_step(dims, U, p, None)
    assert np.array_equal(U1, oracle.step(dims, U, 1)[0])      # s = 1: the plain update
    _, _, d0 = oracle.measure(dims, U)
    P0, c0 = oracle.band_powers(dims, d0)
    assert np.array_equal(x0, mlp.features(P0, c0, V)) and np.array_equal(s1, mlp.factors(p, x0))
    U2, acc, s2, x1 = mlp.learned_step(dims, U1, p, s1)
    cand = mlp.update_with(dims, U1, s1)
    assert np.array_equal(U2, cand if acc else oracle.step(dims, U1, 1)[0])
    Ur, it, fb, F, th = mlp.learned_run(dims, U, p, n=2)
    assert np.array_equal(Ur, U2) and it == 2
def test_linesearch_never_worse_than_plain(oracle_lib):
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 6)
    x, ls, best = mlp.linesearch(dims, U, iters=12)
    th_plain = oracle.measure(dims, oracle.step(dims, U, 1)[0])[1]
    assert best <= th_plain
    assert np.all(np.abs(ls) <= mlp.CLIP + 1e-12)
    assert abs(oracle.measure(dims, mlp.update_with(dims, U, np.exp(ls)))[1] / best - 1) < 1e-12


def test_linesearch_linear_regime_closed_form(oracle_lib):
    """In the linear regime every mode of Delta contracts by
    (1 - alpha p2max s) per update (Fourier acceleration makes the factor the
    same for all momenta), so theta after one update is minimised at
    s = 1 / (alpha p2max) = 1 / 1.28, where it vanishes to first order."""
    dims = (4, 4, 4, 4)
    U = synth.small_field(dims, 9, eps=1e-5)
    x, ls, best = mlp.linesearch(dims, U, iters=24)
    _, _, delta = oracle.measure(dims, U)
    _, cnt = oracle.band_powers(dims, delta)
    target = -np.log(0.08 * 16.0)
    held = cnt > 0
    assert held.sum() >= 3
    assert np.max(np.abs(ls[held] - target)) < 2e-3
    assert np.all(ls[~held] == 0.0)
    th0 = oracle.measure(dims, U)[1]
    assert best < 1e-3 * th0 and oracle.measure(dims, oracle.step(dims, U, 1)[0])[1] > 0.07 * th0


def test_forward_matches_torch_float64():
    """The oracle's network forward against torch's float64 linear layers and
    ReLU on the same bf16-rounded weights and float32 biases, plus the factor
    map s = exp(clip(y, -2.3, 2.3)) written out here."""
    p = random_params(21, scale=0.4)
    rng = np.random.default_rng(22)
    x = rng.normal(size=(64, 16)) * 2.0
    y, _ = mlp.forward(p, x)
    t = {k: torch.from_numpy(np.asarray(v, dtype=np.float64)) for k, v in p.items()}
    h = torch.relu(torch.nn.functional.linear(torch.from_numpy(x), t["W1"].T, t["b1"]))
    h = torch.relu(torch.nn.functional.linear(h, t["W2"].T, t["b2"]))
    yt = torch.nn.functional.linear(h, t["W3"].T, t["b3"]).numpy()
    assert np.max(np.abs(y - yt)) <= 1e-13 * max(1.0, np.max(np.abs(yt)))
    # some outputs must land on each side of the clip, so the map is exercised
    assert np.any(np.abs(yt) > 2.3) and np.any(np.abs(yt) < 2.3)
    for i in range(8):
        s = mlp.factors(p, x[i])
        assert np.max(np.abs(s - np.exp(np.minimum(np.maximum(yt[i], -2.3), 2.3)))) <= 1e-13 * np.max(s)
