"""The library's HIP sources, compiled for the CPU against a stand-in
hip_runtime.h (tests/emu), checked against the FP64 oracle on small lattices.

This runs every kernel's index arithmetic, LDS FFT stages and the runtime's
launch sequencing without a GPU, so layout and bounds mistakes are caught
before a GPU run; the GPU parity tests repeat the comparison on the MI355X.
One case also runs under AddressSanitizer.
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_1206_0675_amd import lgf

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))


@pytest.fixture(scope="module")
def E():
    """The emulated library; LGF_EMU_ASAN=1 selects the AddressSanitizer build
    (run the suite with libasan preloaded)."""
    import build_emu
    return lgf.load_library(build_emu.build(asan=os.environ.get("LGF_EMU_ASAN") == "1"))


CASES = [((4, 4, 4, 4), {}), ((8, 4, 4, 4), {}), ((4, 8, 4, 8), {}), ((4, 4, 16, 4), {}),
         ((16, 16, 4, 4), {}), ((32, 16, 4, 4), {}), ((4, 4, 8, 16), {}),
         ((8, 8, 4, 4), {"storage": 12}), ((4, 4, 4, 8), {"accel": 0})]


@pytest.mark.parametrize("dims, kw", CASES)
def test_emulated_steps_match_oracle(E, oracle_lib, dims, kw):
    U = synth.random_links(dims, 2)
    ctx = lgf.Context(dims, lib=E, **kw)
    ctx.load(U)
    tf, tt = ctx.step(3, trace=True)
    Ug = ctx.store()
    o = oracle.opts(accel=kw.get("accel", 1) == 1, store12=kw.get("storage", 18) == 12)
    Uo, of, ot, _ = oracle.step(dims, U, 3, o)
    assert np.max(np.abs(Ug - Uo)) <= 1e-13
    assert np.max(np.abs(tf - of)) <= 1e-13 * np.max(np.abs(of))
    assert np.max(np.abs(tt / ot - 1)) <= 1e-12


@pytest.mark.parametrize("dims, kw", [((4, 4, 32, 32), {}), ((4, 4, 16, 32), {"storage": 12}),
                                      ((8, 4, 8, 64), {})])
def test_emulated_large_zt_extent_matches_oracle(E, oracle_lib, dims, kw):
    """Many (z, t) planes: the XCD-aware plane order over 8 slabs."""
    U = synth.random_links(dims, 41)
    o = oracle.opts(store12=kw.get("storage", 18) == 12)
    with lgf.Context(dims, lib=E, **kw) as c:
        c.load(U)
        tf, tt = c.step(3, trace=True)
        Ug = c.store()
    Uo, of, ot, _ = oracle.step(dims, U, 3, o)
    assert np.max(np.abs(Ug - Uo)) <= 1e-12
    assert np.max(np.abs(tf - of) / of) <= 1e-12 and np.max(np.abs(tt - ot) / ot) <= 1e-12


def test_emulated_fp32_error_is_single_precision(E, oracle_lib):
    dims = (8, 4, 8, 4)
    U = synth.random_links(dims, 2)
    ctx = lgf.Context(dims, lib=E, precision=lgf.FP32)
    ctx.load(U)
    tf, tt = ctx.step(3, trace=True)
    Uo, of, ot, _ = oracle.step(dims, U, 3)
    d = np.max(np.abs(ctx.store() - Uo))
    assert 1e-9 < d < 1e-5


def test_emulated_fix_and_mixed(E, oracle_lib):
    dims = (4, 4, 8, 4)
    U = synth.random_links(dims, 3)
    _, it, F, th, ok, _ = oracle.fix(dims, U)
    ctx = lgf.Context(dims, lib=E, poll_every=8)
    ctx.load(U)
    s = ctx.fix()
    assert abs(s.iter - it) <= 1 and abs(s.F - F) <= 1e-12 and s.theta < 1e-15
    m = lgf.Context(dims, lib=E, precision=lgf.MIXED, poll_every=8)
    m.load(U)
    s = m.fix()
    assert s.iter_fp32 > 0 and s.iter_fp64 > 0 and s.iter == s.iter_fp32 + s.iter_fp64
    assert abs(s.F - F) <= 1e-9 and s.theta < 1e-15
    G = m.store_gauge()
    assert np.max(np.abs(oracle.transform(dims, U, G) - m.store())) < 1e-12


def test_emulated_mixed_switch_below_the_fp32_floor(E, oracle_lib):
    """theta_switch below anything FP32 can reach: the FP32 phase ends after
    512 updates without theta halving, and FP64 finishes on the oracle's F."""
    dims = (4, 4, 4, 8)
    U = synth.random_links(dims, 3)
    _, it, F, th, ok, _ = oracle.fix(dims, U)
    with lgf.Context(dims, lib=E, precision=lgf.MIXED, storage=12, theta_switch=1e-18) as m:
        m.load(U)
        s = m.fix()
    assert s.status == 0 and s.theta < 1e-15 and s.iter == s.iter_fp32 + s.iter_fp64
    assert s.iter_fp32 >= 512 and 0 < s.iter_fp64 < it
    assert abs(s.F - F) <= 1e-9


def test_emulated_checkpoint_resume(E, oracle_lib):
    """A checkpoint is the loaded links and G: loading both resumes the run
    bit for bit, and the links are G U0 G^dag(x+mu) from the moment G is
    loaded."""
    dims = (4, 8, 4, 4)
    U = synth.random_links(dims, 4)
    a = lgf.Context(dims, lib=E)
    a.load(U)
    a.step(4)
    U4, G4 = a.store(), a.store_gauge()
    a.step(3)
    ref = a.store()
    b = lgf.Context(dims, lib=E)
    b.load(U)
    b.load_gauge(G4)
    assert np.array_equal(b.store(), U4)
    assert np.max(np.abs(oracle.transform(dims, U, G4) - U4)) <= 1e-13
    b.step(3)
    assert np.array_equal(b.store(), ref)
    assert np.max(np.abs(b.store_gauge() - a.store_gauge())) == 0.0


def test_emulated_load_rejects_bad_links(E):
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 1)
    ctx = lgf.Context(dims, lib=E)
    bad = U.copy()
    bad[0, 0, 0, 0, 0] *= 1.001
    with pytest.raises(lgf.LgfError) as e:
        ctx.load(bad)
    assert e.value.code == lgf.E_NOT_UNITARY
    with pytest.raises(lgf.LgfError) as e:
        ctx.step(1)
    assert e.value.code == lgf.E_STATE
    bad[0, 0, 0, 0, 0, 0, 0] = np.inf
    with pytest.raises(lgf.LgfError) as e:
        ctx.load(bad)
    assert e.value.code == lgf.E_NONFINITE


_ASAN_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import synth
from paper_1206_0675_amd import lgf
L = lgf.load_library({lib!r})
for dims, kw in [((4, 4, 4, 4), {{"max_iter": 4}}), ((8, 4, 4, 8), {{"storage": 12, "max_iter": 4}}),
                 ((4, 8, 4, 4), {{"precision": 2, "poll_every": 4, "theta_switch": 1.0, "max_iter": 8}}),
                 ((4, 4, 8, 4), {{"precision": 1, "max_iter": 4}}),
                 ((4, 4, 32, 32), {{"storage": 12, "max_iter": 3}}),
                 ((16, 8, 4, 4), {{"storage": 12, "autotune": 1, "max_iter": 3}})]:
    ctx = lgf.Context(dims, lib=L, **kw)
    ctx.load(synth.random_links(dims, 5))
    ctx.step(2, trace=True)
    ctx.fix(raise_on_error=False)
    ctx.store()
    ctx.load_gauge(ctx.store_gauge())
    ctx.close()
print("ASAN-CLEAN")
"""


@pytest.mark.slow
def test_emulated_under_address_sanitizer():
    import build_emu
    lib = build_emu.build(asan=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0")
    root = os.path.dirname(HERE)
    r = subprocess.run([sys.executable, "-c", _ASAN_SCRIPT.format(root=root, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "ASAN-CLEAN" in r.stdout, r.stderr[-3000:]


def test_emulated_batch_members_match_oracle(E, oracle_lib):
    dims = [(4, 4, 4, 4), (8, 4, 4, 8), (4, 8, 4, 4)]
    Us = [synth.random_links(d, 20 + i) for i, d in enumerate(dims)]
    with lgf.Batch(dims, lib=E, poll_every=4) as b:
        for i, U in enumerate(Us):
            b.load(i, U)
        st = b.fix()
        for i, (d, U) in enumerate(zip(dims, Us)):
            _, it, F, th, ok, _ = oracle.fix(d, U)
            assert st[i].status == lgf.OK and abs(st[i].iter - it) <= 1 and abs(st[i].F - F) <= 1e-12
            Uo, _, _, _ = oracle.step(d, U, st[i].iter)
            assert np.max(np.abs(b.store(i) - Uo)) <= 1e-12


def test_emulated_batch_mixed_autotuned(E, oracle_lib):
    dims = [(4, 4, 4, 4), (4, 4, 8, 4)]
    Us = [synth.random_links(d, 30 + i, eps=0.2 + 0.2 * i) for i, d in enumerate(dims)]
    with lgf.Batch(dims, lib=E, precision=lgf.MIXED, storage=12, poll_every=4, autotune=1) as b:
        nth, tb = b.config()
        assert nth in (64, 128, 256) and tb in (32, 64, 128)
        for i, U in enumerate(Us):
            b.load(i, U)
        st = b.fix()
        for i, (d, U) in enumerate(zip(dims, Us)):
            _, it, F, th, ok, _ = oracle.fix(d, U)
            assert st[i].status == lgf.OK and st[i].iter_fp32 > 0 and st[i].iter_fp64 > 0
            assert abs(st[i].F - F) <= 1e-9 and st[i].theta < 1e-15
            G = b.store_gauge(i)
            assert np.max(np.abs(oracle.transform(d, U, G) - b.store(i))) <= 1e-12
    outs, sts, rc = lgf.fix_batch(Us, lib=E, poll_every=4)
    assert rc == lgf.OK and all(s.theta < 1e-15 for s in sts)


def test_emulated_single_autotune_and_forced_shapes(E, oracle_lib, tmp_path, monkeypatch):
    """lgf_params.autotune on a single lattice picks one of the candidate
    launch shapes and caches it; a cached shape is taken as is; every shape
    gives bit-identical links (the arithmetic per element does not depend on
    the launch shape), equal to the oracle's."""
    dims = (16, 8, 4, 4)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LGF_TUNE_CACHE", str(cache))
    U = synth.random_links(dims, 5)
    with lgf.Context(dims, lib=E, storage=12, autotune=1) as c:
        picked = c.config()
    key, nth, tb = cache.read_text().split()
    assert (int(nth), int(tb)) == picked and picked[0] in (64, 128) and picked[1] in (32, 64, 128)
    Uo = oracle.step(dims, U, 3)[0]
    ref = None
    for shape in [(n, t) for n in (64, 128) for t in (32, 64, 128)]:
        cache.write_text(f"{key} {shape[0]} {shape[1]}\n")
        with lgf.Context(dims, lib=E, storage=12, autotune=1) as c:
            assert c.config() == shape
            c.load(U)
            c.step(3)
            out = c.store()
        assert np.max(np.abs(out - Uo)) <= 1e-12
        if ref is None:
            ref = out
        assert np.array_equal(out, ref), shape
    with lgf.Context(dims, lib=E, storage=12) as c:
        assert c.config() == (128, 128)


# ---------------------------------------------------------------------------
# learned spectral step (FP64) and the network kernels
# ---------------------------------------------------------------------------
from oracle import mlp as omlp  # noqa: E402


def _rand_blob(seed, scale=0.3, b3=None):
    rng = np.random.default_rng(seed)
    p = {k: rng.normal(scale=scale, size=s) for k, s in omlp.SHAPES}
    if b3 is not None:
        p["b3"] = np.full(16, b3)
    return omlp.blob_from_params(p)


def test_emulated_learned_zero_model_is_plain(E, oracle_lib):
    dims = (4, 4, 8, 4)
    U = synth.random_links(dims, 7)
    zero = omlp.blob_from_params({k: np.zeros(s) for k, s in omlp.SHAPES})
    with lgf.Context(dims, lib=E, step=1) as a, lgf.Context(dims, lib=E) as b:
        a.set_model(zero)
        a.load(U)
        b.load(U)
        fa, ta = a.step(3, trace=True)
        fb, tb = b.step(3, trace=True)
        assert np.array_equal(a.store(), b.store()) and np.array_equal(fa, fb)


def test_emulated_learned_factors_and_update_match_oracle(E, oracle_lib):
    """Features and factors before each of three updates against the oracle;
    the links after each update equal the oracle's update with the factors the
    library applied (s = 1 first, then the network's factors of the previous
    spectrum) and its accept rule."""
    dims = (8, 4, 4, 8)
    V = synth.volume(dims)
    U = synth.random_links(dims, 8)
    blob = _rand_blob(9, scale=0.2)
    p = omlp.params_from_blob(blob)
    Uo, s_use = U, np.ones(16)
    with lgf.Context(dims, lib=E, step=1) as c:
        c.set_model(blob)
        c.load(U)
        for _ in range(3):
            x, s_next = c.learned_factors()
            F0, th0, delta = oracle.measure(dims, Uo)
            P, cnt = oracle.band_powers(dims, delta)
            xo = omlp.features(P, cnt, V)
            assert np.max(np.abs(x - xo)) <= 1e-12
            assert np.max(np.abs(s_next / omlp.factors(p, xo) - 1)) <= 1e-5
            c.step(1)
            Uc = omlp.update_with(dims, Uo, s_use)
            F1, th1, _ = oracle.measure(dims, Uc)
            Uo = Uc if (F1 > F0 or th1 < th0) else oracle.step(dims, Uo, 1)[0]
            assert np.max(np.abs(c.store() - Uo)) <= 1e-12
            s_use = s_next


def test_emulated_learned_steps_trace_match_oracle(E, oracle_lib):
    """Four learned updates queued back to back (the accept decision and the
    next factors made on the device) equal, bitwise, four single updates, and
    follow the oracle's lagged learned run: the fallback count matches and F,
    theta at the end agree."""
    dims = (4, 8, 4, 4)
    U = synth.random_links(dims, 14)
    blob = _rand_blob(15, scale=0.2, b3=0.3)
    p = omlp.params_from_blob(blob)
    with lgf.Context(dims, lib=E, step=1) as c:
        c.set_model(blob)
        c.load(U)
        tf, tt = c.step(4, trace=True)
        Ug = c.store()
        fb = c.measure().fallbacks
    with lgf.Context(dims, lib=E, step=1) as c:
        c.set_model(blob)
        c.load(U)
        for _ in range(4):
            c.step(1)
        assert np.array_equal(c.store(), Ug)
    Uo, it, rejected, Fo, tho = omlp.learned_run(dims, U, p, n=4)
    assert np.max(np.abs(Ug - Uo)) <= 1e-6      # the network's factors differ by ~1e-7 (float32)
    assert fb == rejected
    assert abs(tf[-1] - Fo) <= 1e-7 and abs(tt[-1] / tho - 1) <= 1e-4


@pytest.mark.parametrize("poll", [2])
def test_emulated_learned_fix_graph_matches_eager(E, poll):
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 16)
    blob = _rand_blob(17, scale=0.0, b3=1.2)      # s = 3.3: rejected once the run is near-linear
    out = []
    for kw in (dict(poll_every=poll), dict(poll_every=poll, no_graph=1)):
        with lgf.Context(dims, lib=E, step=1, max_iter=400, theta_stop=1e-6, **kw) as c:
            c.set_model(blob)
            c.load(U)
            c.step(1)                       # odd number of Delta-buffer swaps before the graph
            st = c.fix()
            out.append((c.store(), st.iter, st.fallbacks, st.F))
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2] and out[0][3] == out[1][3]
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][2] > 0                            # fallbacks inside captured chunks


def test_emulated_mlp_kernels_match_oracle(E):
    blob = _rand_blob(10)
    p = omlp.params_from_blob(blob)
    rng = np.random.default_rng(11)
    X, T = rng.normal(size=(40, 16)), rng.normal(size=(40, 16))
    M = (rng.random((40, 16)) > 0.25).astype(float)
    Y = lgf.mlp_eval(blob, X, lib=E)
    Yo, _ = omlp.forward(p, X.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(Y - Yo)) <= 1e-5 * max(1.0, np.max(np.abs(Yo)))
    loss, g = lgf.mlp_grad(blob, X, T, M, lib=E)
    lo, go = omlp.loss_and_grad(p, X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64), M)
    go = omlp.flat(go)
    assert abs(loss - lo) <= 1e-5 * lo
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)


def test_emulated_mlp_training_reduces_loss(E):
    rng = np.random.default_rng(12)
    X = rng.normal(size=(512, 16)) * 0.5
    T = np.tanh(X @ rng.normal(size=(16, 16)) * 0.3)
    M = np.ones_like(X)
    blob, trace = lgf.mlp_train(X, T, M, steps=300, batch=64, seed=3, lr=3e-3, lib=E)
    p = omlp.params_from_blob(blob)
    l_end = omlp.loss_and_grad(p, X, T, M)[0]
    assert trace[-20:].mean() < 0.5 * trace[:5].mean() and l_end < 0.5 * trace[0]


def test_emulated_linesearch_matches_oracle(E, oracle_lib):
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 13)
    with lgf.Context(dims, lib=E) as c:
        c.load(U)
        x, ls = c.linesearch_bands()
        assert np.array_equal(c.store(), U)          # the links are not changed
    xo, lso, best = omlp.linesearch(dims, U)
    assert np.max(np.abs(x - xo)) <= 1e-12
    # both searches end in the same minimum of theta (they may split at
    # near-ties, so compare theta at the chosen factors, not the factors)
    thg = oracle.measure(dims, omlp.update_with(dims, U, np.exp(ls)))[1]
    assert abs(thg / best - 1) <= 1e-6
    assert thg < oracle.measure(dims, oracle.step(dims, U, 1)[0])[1]


# ---------------------------------------------------------------------------
# Wilson-action generator
# ---------------------------------------------------------------------------
from oracle import wilson as owil  # noqa: E402


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 4)])
def test_emulated_wilson_generator_matches_oracle(E, oracle_lib, dims):
    """Heatbath, overrelaxation and a generate run of the library (emulated)
    against the reference.  The library keeps rows 0 and 1 of each link and
    rebuilds row 2, so the first sweep from loaded links sees them to
    rounding; every later sweep starts from SU(3)-projected links, whose row
    2 is rebuilt to the last bit, and agrees with the reference exactly (same
    libm on the CPU)."""
    U = synth.random_links(dims, 3) if dims == (4, 4, 4, 4) else owil.cold(dims)
    with lgf.WilsonGenerator(dims, 5.9, 77, lib=E) as g:
        g.load(U)
        assert np.array_equal(g.store(), U)
        g.sweep(lgf.HEATBATH)
        Uo, sk = owil.sweep(dims, U, 5.9, 77, 0, owil.HEATBATH)
        Ug = g.store()
        assert np.max(np.abs(Ug - Uo)) <= 1e-13 and g.skipped() == sk == 0
        assert g.sweep_index == 1
        g.sweep(lgf.OVERRELAX)
        Uo, _ = owil.sweep(dims, Ug, 5.9, 77, 0, owil.OVERRELAX)
        assert np.array_equal(g.store(), Uo)
        g.update(2, 2)
        Uo, _ = owil.generate(dims, Uo, 5.9, 77, 1, 2, 2)
        assert np.array_equal(g.store(), Uo)
        # the hand-off buffer (emulated device memory is host memory) is
        # rewritten from the sweeps' even-odd copy
        g.sweep(lgf.OVERRELAX)
        Uo, _ = owil.sweep(dims, Uo, 5.9, 77, 3, owil.OVERRELAX)
        n = 2 * Uo.size
        Ud = np.ctypeslib.as_array((ctypes.c_double * n).from_address(g.device_links))
        assert np.max(np.abs(Ud.view(np.complex128).reshape(Uo.shape) - Uo)) <= 1e-13
        if dims == (4, 4, 4, 4):
            assert abs(g.plaquette() - oracle.plaquette(dims, Uo)) <= 1e-14
        g.cold()
        assert g.sweep_index == 0 and np.array_equal(g.store(), owil.cold(dims))


def test_emulated_wilson_small_beta_and_errors(E, oracle_lib):
    """beta < 3/k runs the plain-rejection branch of the x0 sampler; invalid
    arguments are refused."""
    dims = (4, 4, 2, 2)
    with lgf.WilsonGenerator(dims, 0.2, 5, lib=E) as g:
        g.update(2, 1)
        Uo, sk = owil.generate(dims, owil.cold(dims), 0.2, 5, 0, 2, 1)
        assert np.max(np.abs(g.store() - Uo)) <= 1e-13 and g.skipped() == sk == 0
        with pytest.raises(lgf.LgfError):
            g.sweep(7)
    for bad in ((3, 4, 4, 4), (4, 4, 4, 0)):
        with pytest.raises(lgf.LgfError):
            lgf.WilsonGenerator(bad, 6.0, 1, lib=E)
    with pytest.raises(lgf.LgfError):
        lgf.WilsonGenerator((4, 4, 4, 4), -1.0, 1, lib=E)


# ---------------------------------------------------------------------------
# FFT decomposition study
# ---------------------------------------------------------------------------
def _pack(D):
    """(..., 3, 3) Delta -> the four complex fields (4, ...) the filter runs on."""
    return np.ascontiguousarray(np.stack([D[..., 0, 1], D[..., 0, 2], D[..., 1, 2],
                                          D[..., 0, 0].imag + 1j * D[..., 1, 1].imag]))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 16, 4), (4, 8, 4, 8), (4, 4, 4, 16), (4, 4, 4, 32)])
def test_emulated_fft_study_matches_oracle_filter(E, oracle_lib, dims):
    """The decompositions apply the oracle's filter (K real and even, so
    filtering the packed fields is the packed filter of Delta); the matrix-core
    t pass runs for Lt >= 16."""
    U = synth.random_links(dims, 2)
    _, _, delta = oracle.measure(dims, U)
    ref = _pack(oracle.filter_delta(dims, delta))
    f = _pack(delta)
    variants = [lgf.FFT_1DX4, lgf.FFT_2D1D1D, lgf.FFT_2D2D] + ([lgf.FFT_2D1D1D_MFMA] if dims[3] >= 16 else [])
    for v in variants:
        out, _ = lgf.fft_study(dims, v, f, lib=E)
        assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref)), v
    with pytest.raises(lgf.LgfError):
        lgf.fft_study((4, 4, 4, 128), 0, np.zeros((4, 128, 4, 4, 4), complex), lib=E)
    with pytest.raises(lgf.LgfError):
        lgf.fft_study(dims, 4, f, lib=E)


@pytest.mark.parametrize("dims, kw", [((8, 8, 8, 8), {}), ((8, 8, 8, 8), {"precision": 2, "storage": 12}),
                                      ((4, 8, 4, 8), {"poll_every": 4})])
def test_emulated_captured_chunks_equal_single_updates(E, dims, kw):
    """In a captured chunk each update's reduction runs in the next update's
    (z, t) launch; the run must equal the one launched update by update, bit
    for bit, and leave a context that measures the same."""
    U = synth.random_links(dims, 5)
    res = []
    for ng in (0, 1):
        with lgf.Context(dims, lib=E, no_graph=ng, **kw) as c:
            c.load(U)
            s = c.fix()
            m = c.measure()
            res.append((s.iter, s.F, s.theta, c.store(), m.F, m.theta))
    a, b = res
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2] and np.array_equal(a[3], b[3])
    assert a[4] == b[4] and a[5] == b[5]
