"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed
form, a library routine (numpy.fft, scipy.linalg.expm), brute force, a
finite difference, or an invariant of the method (gauge invariance of the
plaquette, ascent of F).  Together they are chosen so that a dropped term, a
wrong sign, a wrong neighbour index or a transposed operand in the oracle
fails at least one of them.
"""
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth

ALPHA = 0.08


def dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def fwd(a, mu, step=1):
    """b[x] = a[x + step*mu] on an array whose leading axes are (t, z, y, x)."""
    return np.roll(a, -step, axis=3 - mu)


def np_plaquette(U):
    """Mean plaquette written independently of the oracle (numpy)."""
    acc = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = U[..., mu, :, :]
            b = fwd(U[..., nu, :, :], mu)
            c = fwd(U[..., mu, :, :], nu)
            d = U[..., nu, :, :]
            p = a @ b @ dag(c) @ dag(d)
            acc += np.real(np.trace(p, axis1=-2, axis2=-1)).sum()
    return acc / (18.0 * U[..., 0, 0, 0].size)


def phat2(dims, n):
    return sum(4 * np.sin(np.pi * n[m] / dims[m]) ** 2 for m in range(4))


def coords(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return (x, y, z, t)


# --------------------------------------------------------------------------
# P-1  U = 1: Delta = 0, theta = 0, F = 1, and an update is a no-op (exact)
# --------------------------------------------------------------------------
def test_identity_is_fixed_point(oracle_lib):
    dims = (4, 4, 4, 4)
    U = synth.identity_links(dims)
    F, th, d = oracle.measure(dims, U)
    assert F == 1.0 and th == 0.0 and np.all(d == 0)
    U2, tf, tt, _ = oracle.step(dims, U, 3)
    assert np.array_equal(U2, U)
    assert np.all(tf == 1.0) and np.all(tt == 0.0)


# --------------------------------------------------------------------------
# F and theta normalisation on fields with closed-form values (Section 2)
# --------------------------------------------------------------------------
def test_F_constant_field_closed_form(oracle_lib):
    dims = (4, 2, 4, 2)
    phi = 0.7
    U = synth.identity_links(dims)
    U[..., :, :, :] = np.diag([np.exp(1j * phi), np.exp(-1j * phi), 1.0])
    F, th, _ = oracle.measure(dims, U)
    assert abs(F - (2 * np.cos(phi) + 1) / 3) < 1e-15
    assert th == 0.0                      # a constant field is in Landau gauge


def test_theta_closed_form_abelian_x_wave(oracle_lib):
    # U_x(x) = diag(e^{i phi(x)}, e^{-i phi(x)}, 1), other links 1:
    # Delta_00 = 2i (sin phi(x-1) - sin phi(x)) = -Delta_11, Delta_22 = 0,
    # so |Delta|^2 = 8 (sin phi(x-1) - sin phi(x))^2 and theta = sum / (3V).
    dims = (8, 2, 2, 2)
    V = synth.volume(dims)
    rng = np.random.default_rng(3)
    phi_x = rng.uniform(-1, 1, size=8)
    U = synth.identity_links(dims)
    for x in range(8):
        U[:, :, :, x, 0] = np.diag([np.exp(1j * phi_x[x]), np.exp(-1j * phi_x[x]), 1.0])
    F, th, d = oracle.measure(dims, U)
    diff = np.sin(np.roll(phi_x, 1)) - np.sin(phi_x)
    expect = 8 * np.sum(diff ** 2) * (V // 8) / (3 * V)
    assert abs(th - expect) <= 1e-14 * expect
    assert np.allclose(d[0, 0, 0, :, 0, 0], 2j * diff, atol=1e-15)
    assert np.allclose(d[0, 0, 0, :, 1, 1], -2j * diff, atol=1e-15)
    Fexp = (np.sum(2 * np.cos(phi_x) + 1) / 8 + 3 * 3) / 12
    assert abs(F - Fexp) < 1e-15


# --------------------------------------------------------------------------
# P-6  FFT against numpy.fft and against the brute-force DFT
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 4, 2), (2, 8, 2, 4)])
def test_fft_matches_numpy(oracle_lib, dims):
    rng = np.random.default_rng(1)
    shape = (dims[3], dims[2], dims[1], dims[0])
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    fw = oracle.fft4d(dims, f, -1)
    ref = np.fft.fftn(f)
    assert np.max(np.abs(fw - ref)) <= 1e-13 * np.max(np.abs(ref))
    bw = oracle.fft4d(dims, f, +1)
    refb = np.fft.ifftn(f) * f.size
    assert np.max(np.abs(bw - refb)) <= 1e-13 * np.max(np.abs(refb))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 4)])
def test_fft_matches_bruteforce_dft(oracle_lib, dims):
    rng = np.random.default_rng(2)
    shape = (dims[3], dims[2], dims[1], dims[0])
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    xs = np.stack([c.ravel() for c in coords(dims)], axis=1)          # (V, 4)
    phase = sum(np.outer(xs[:, m], xs[:, m]) / dims[m] for m in range(4))
    dft = np.exp(-2j * np.pi * phase)
    ref = (dft @ f.ravel()).reshape(shape)
    got = oracle.fft4d(dims, f, -1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# P-9  a plane wave is an eigenvector of the acceleration: eigenvalue K(n)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [(1, 0, 0, 0), (1, 2, 0, 3), (4, 4, 4, 4), (0, 0, 7, 1)])
def test_filter_plane_wave_eigenvalue(oracle_lib, n):
    dims = (8, 8, 8, 8)
    x = coords(dims)
    phase = np.exp(2j * np.pi * sum(n[m] * x[m] / dims[m] for m in range(4)))
    M = np.arange(9).reshape(3, 3) * (0.3 + 0.1j) - 1.0
    delta = phase[..., None, None] * M
    out = oracle.filter_delta(dims, delta)
    K = 16.0 / phat2(dims, n)
    assert np.max(np.abs(out - K * delta)) <= 1e-13 * K * np.max(np.abs(delta))
    plain = oracle.filter_delta(dims, delta, oracle.opts(accel=False))
    assert np.max(np.abs(plain - delta)) <= 1e-13 * np.max(np.abs(delta))


def test_filter_zero_mode_removed(oracle_lib):
    dims = (4, 4, 4, 4)
    delta = np.ones((4, 4, 4, 4, 3, 3), dtype=np.complex128)
    assert np.max(np.abs(oracle.filter_delta(dims, delta))) < 1e-15


# --------------------------------------------------------------------------
# g(x): first order in alpha, then projection to SU(3) by row Gram-Schmidt
# --------------------------------------------------------------------------
def test_gauge_projection_properties(oracle_lib):
    dims = (4, 4, 2, 2)
    rng = np.random.default_rng(5)
    shape = (2, 2, 4, 4, 3, 3)
    H = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    D = H - dag(H)
    D -= np.trace(D, axis1=-2, axis2=-1)[..., None, None] / 3 * np.eye(3)
    g = oracle.gauge(dims, D, ALPHA)
    M = np.eye(3) + 0.5 * ALPHA * D
    # in SU(3)
    assert np.max(np.abs(g @ dag(g) - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(g) - 1)) < 1e-14
    # row 1 of g is row 1 of M normalised; row 2 lies in span(row 1, row 2 of M)
    r0 = M[..., 0, :] / np.linalg.norm(M[..., 0, :], axis=-1)[..., None]
    assert np.max(np.abs(g[..., 0, :] - r0)) < 1e-15
    P = np.stack([M[..., 0, :], M[..., 1, :]], axis=-2)                   # (...,2,3)
    coef, *_ = zip(*[np.linalg.lstsq(P.reshape(-1, 2, 3)[i].T, g.reshape(-1, 3, 3)[i, 1], rcond=None)
                     for i in range(P.reshape(-1, 2, 3).shape[0])])
    resid = [np.linalg.norm(P.reshape(-1, 2, 3)[i].T @ c - g.reshape(-1, 3, 3)[i, 1])
             for i, c in enumerate(coef)]
    assert max(resid) < 1e-14
    # first order in alpha: g agrees with exp(alpha/2 D) up to O(alpha^2 |D|^2)
    E = scipy.linalg.expm(0.5 * ALPHA * D.reshape(-1, 3, 3)).reshape(shape)
    err = np.max(np.abs(g - E))
    assert err < 0.5 * (0.5 * ALPHA * np.max(np.abs(D))) ** 2 * 9


def test_gauge_fixes_su3_points(oracle_lib):
    # if 1 + alpha/2 d is already in SU(3) the projection returns it unchanged
    dims = (2, 2, 2, 2)
    W = synth.haar_su3(11, 16).reshape(2, 2, 2, 2, 3, 3)
    d = (W - np.eye(3)) * (2.0 / ALPHA)
    g = oracle.gauge(dims, d, ALPHA)
    assert np.max(np.abs(g - W)) < 1e-14


# --------------------------------------------------------------------------
# transform: group action and gauge invariance (P-2)
# --------------------------------------------------------------------------
def test_transform_is_group_action(oracle_lib):
    dims = (4, 4, 4, 2)
    U = synth.random_links(dims, 3)
    g1 = synth.haar_su3(21, synth.volume(dims)).reshape(2, 4, 4, 4, 3, 3)
    g2 = synth.haar_su3(22, synth.volume(dims)).reshape(2, 4, 4, 4, 3, 3)
    a = oracle.transform(dims, oracle.transform(dims, U, g1), g2)
    b = oracle.transform(dims, U, g2 @ g1)
    assert np.max(np.abs(a - b)) < 1e-14
    # constant g = C: U -> C U C^dagger link by link
    C = synth.haar_su3(23, 1)[0]
    c = oracle.transform(dims, U, np.broadcast_to(C, g1.shape).copy())
    assert np.max(np.abs(c - C @ U @ dag(C))) < 1e-14
    # the orbit of 1 is h(x) h^dagger(x+mu)
    one = synth.identity_links(dims)
    pg = oracle.transform(dims, one, g1)
    for mu in range(4):
        assert np.max(np.abs(pg[..., mu, :, :] - g1 @ dag(fwd(g1, mu)))) < 1e-15


def test_plaquette_matches_numpy_and_is_gauge_invariant(oracle_lib):
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 4)
    p = oracle.plaquette(dims, U)
    assert abs(p - np_plaquette(U)) < 1e-14
    g = synth.haar_su3(31, synth.volume(dims)).reshape(4, 4, 4, 4, 3, 3)
    assert abs(oracle.plaquette(dims, oracle.transform(dims, U, g)) - p) < 1e-13


def test_plaquette_invariant_along_fix(oracle_lib):
    dims = (8, 8, 8, 8)
    U = synth.random_links(dims, 1)
    p0 = oracle.plaquette(dims, U)
    U2, it, F, th, ok, _ = oracle.fix(dims, U)
    assert ok and th < 1e-15
    assert abs(oracle.plaquette(dims, U2) - p0) < 1e-12
    assert abs(np_plaquette(U2) - p0) < 1e-12


# --------------------------------------------------------------------------
# P-7  Delta is the gradient of F: dF/dh along exp(hX) at one site
# --------------------------------------------------------------------------
def test_delta_is_gradient_of_F(oracle_lib):
    dims = (4, 4, 4, 4)
    V = synth.volume(dims)
    U = synth.random_links(dims, 5)
    _, _, delta = oracle.measure(dims, U)
    rng = np.random.default_rng(7)
    site = (1, 2, 3, 0)                      # (t, z, y, x) array index
    A = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    X = A - dag(A)
    X -= np.trace(X) / 3 * np.eye(3)

    def F_at(h):
        g = synth.identity_links((4, 4, 4, 4))[..., 0, :, :].copy()
        g[site] = scipy.linalg.expm(h * X)
        return oracle.measure(dims, oracle.transform(dims, U, g))[0]

    h = 1e-4
    fd = (F_at(h) - F_at(-h)) / (2 * h)
    an = -np.real(np.trace(X @ delta[site])) / (24 * V)
    assert abs(fd - an) <= 1e-6 * abs(an)


# --------------------------------------------------------------------------
# P-11  sum_x Delta(x) = 0 (periodic telescoping); Delta anti-Hermitian traceless
# --------------------------------------------------------------------------
def test_delta_sum_zero_and_algebra(oracle_lib):
    dims = (8, 4, 4, 4)
    U = synth.random_links(dims, 6)
    _, _, d = oracle.measure(dims, U)
    s = d.reshape(-1, 3, 3).sum(axis=0)
    assert np.max(np.abs(s)) <= 1e-13 * synth.volume(dims) * np.max(np.abs(d))
    assert np.max(np.abs(d + dag(d))) < 1e-15
    assert np.max(np.abs(np.trace(d, axis1=-2, axis2=-1))) < 1e-14


# --------------------------------------------------------------------------
# P-8  linearised contraction: theta_1/theta_0 = (1 - alpha p2max)^2 = 0.0784
#       and, without acceleration, (1 - alpha p^2(n))^2 for a plane wave
# --------------------------------------------------------------------------
def test_linear_regime_contraction_small_field(oracle_lib):
    dims = (8, 8, 8, 8)
    U = synth.small_field(dims, 9, eps=1e-5)
    _, _, tt, _ = oracle.step(dims, U, 1)
    assert abs(tt[1] / tt[0] - (1 - 16 * ALPHA) ** 2) <= 1e-4 * 0.0784


def _abelian_wave(dims, n, eps):
    x = coords(dims)
    c = (1.0, 0.5, -0.7, 0.3)
    ph = 2 * np.pi * sum(n[m] * x[m] / dims[m] for m in range(4))
    U = synth.identity_links(dims)
    for mu in range(4):
        a = eps * c[mu] * np.cos(ph + 0.4 * mu)          # A_mu = a * lambda_3 / 2
        U[..., mu, 0, 0] = np.exp(0.5j * a)
        U[..., mu, 1, 1] = np.exp(-0.5j * a)
    return U


@pytest.mark.parametrize("n", [(1, 2, 0, 3), (1, 0, 0, 0), (2, 2, 2, 2)])
def test_linear_regime_plane_wave(oracle_lib, n):
    dims = (8, 8, 8, 8)
    U = _abelian_wave(dims, n, 1e-6)
    _, _, tt, _ = oracle.step(dims, U, 1, oracle.opts(accel=False))
    expect = (1 - ALPHA * phat2(dims, n)) ** 2
    assert abs(tt[1] / tt[0] - expect) <= 1e-8
    _, _, ta, _ = oracle.step(dims, U, 1)
    assert abs(ta[1] / ta[0] - (1 - 16 * ALPHA) ** 2) <= 1e-8


# --------------------------------------------------------------------------
# P-3, P-4, P-5  ascent, the orbit of 1, unitarity
# --------------------------------------------------------------------------
def test_F_monotone_and_fix_stops_at_threshold(oracle_lib):
    dims = (8, 8, 8, 8)
    U = synth.random_links(dims, 1)
    _, tf, tt, _ = oracle.step(dims, U, 40)
    assert np.all(np.diff(tf) >= -1e-14)
    U2, it, F, th, ok, _ = oracle.fix(dims, U)
    assert ok and th < 1e-15
    assert tt[it - 1] >= 1e-15 and tt[it] < 1e-15
    assert F == tf[it] and th == tt[it]
    mu, md = oracle.unitarity(U2)
    assert mu < 1e-12 and md < 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pure_gauge_converges_to_F_one(oracle_lib, seed):
    dims = (4, 4, 4, 4)
    U = synth.pure_gauge(dims, seed)
    U2, it, F, th, ok, _ = oracle.fix(dims, U)
    assert ok and th < 1e-15
    assert abs(F - 1.0) <= 1e-12
    assert np.max(np.abs(U2 - np.eye(3))) < 1e-6     # the links become a constant C: here ~1


def test_g_field_in_su3(oracle_lib):
    dims = (8, 4, 4, 4)
    U = synth.random_links(dims, 8)
    _, _, d = oracle.measure(dims, U)
    g = oracle.gauge(dims, oracle.filter_delta(dims, d), ALPHA)
    mu, md = oracle.unitarity(g)
    assert mu < 1e-14 and md < 1e-14


# --------------------------------------------------------------------------
# P-10  covariance: translation and axis permutation act on whole
#       trajectories; a constant colour rotation C acts on Delta, F, theta and
#       the filtered field.  (Row Gram-Schmidt does not commute with C at
#       O(alpha^2 |dtilde|^2), so whole trajectories are not C-invariant.)
# --------------------------------------------------------------------------
def test_covariance_translation_and_permutation(oracle_lib):
    dims = (8, 8, 8, 8)
    U = synth.random_links(dims, 12)
    _, tf, tt, _ = oracle.step(dims, U, 6)
    Ut = np.roll(np.roll(U, 3, axis=3), -1, axis=0)
    _, tf2, tt2, _ = oracle.step(dims, Ut, 6)
    Up = np.swapaxes(U, 2, 3)[..., [1, 0, 2, 3], :, :].copy()      # swap x <-> y
    _, tf3, tt3, _ = oracle.step(dims, Up, 6)
    Uq = np.swapaxes(U, 0, 1)[..., [0, 1, 3, 2], :, :].copy()      # swap z <-> t
    _, tf4, tt4, _ = oracle.step(dims, Uq, 6)
    for a, b in [(tf2, tt2), (tf3, tt3), (tf4, tt4)]:
        assert np.max(np.abs(a - tf)) <= 1e-13
        assert np.max(np.abs(b - tt) / tt) <= 1e-11


def test_covariance_constant_colour_rotation(oracle_lib):
    dims = (8, 4, 4, 8)
    U = synth.random_links(dims, 16)
    C = synth.haar_su3(40, 1)[0]
    F, th, d = oracle.measure(dims, U)
    F1, th1, d1 = oracle.measure(dims, C @ U @ dag(C))
    assert abs(F1 - F) < 1e-14 and abs(th1 - th) < 1e-13 * th
    assert np.max(np.abs(d1 - C @ d @ dag(C))) < 1e-13
    f, f1 = oracle.filter_delta(dims, d), oracle.filter_delta(dims, d1)
    assert np.max(np.abs(f1 - C @ f @ dag(C))) < 1e-12


# --------------------------------------------------------------------------
# P-12  12-real storage (third row rebuilt) gives the 18-real trajectory
# --------------------------------------------------------------------------
def test_store12_equals_store18(oracle_lib):
    dims = (8, 8, 4, 4)
    U = synth.random_links(dims, 13)
    U18, f18, t18, _ = oracle.step(dims, U, 10)
    U12, f12, t12, _ = oracle.step(dims, U, 10, oracle.opts(store12=True))
    assert np.max(np.abs(U12 - U18)) <= 1e-13
    assert np.max(np.abs(f12 - f18)) <= 1e-13
    assert np.max(np.abs(t12 - t18) / t18) <= 1e-12


def test_rebuild_row3_is_exact_on_su3(oracle_lib):
    W = synth.haar_su3(50, 1000)
    assert np.max(np.abs(oracle.rebuild_row3(W) - W)) < 1e-15


# --------------------------------------------------------------------------
# P-16  accumulated gauge: U_n = G U_0 G^dagger(x+mu)
# --------------------------------------------------------------------------
def test_accumulated_gauge_reproduces_links(oracle_lib):
    dims = (8, 4, 4, 4)
    U = synth.random_links(dims, 14)
    Un, _, _, G = oracle.step(dims, U, 12, want_G=True)
    assert np.max(np.abs(oracle.transform(dims, U, G) - Un)) < 1e-12
    mu, md = oracle.unitarity(G)
    assert mu < 1e-13 and md < 1e-13


# --------------------------------------------------------------------------
# P-13  generator: calibrated plaquette, Haar moments
# --------------------------------------------------------------------------
def test_generator_plaquette_and_haar_moments(oracle_lib):
    dims = (8, 8, 8, 8)
    U = synth.random_links(dims, 1)
    assert abs(oracle.plaquette(dims, U) - 0.600) < 0.005
    g = synth.haar_su3(77, 200000)
    tr = np.trace(g, axis1=1, axis2=2)
    assert abs(np.mean(tr)) < 3 * np.sqrt(1 / 200000) * 1.5
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 3 * np.sqrt(1 / 200000) * 1.5 * 1.5
    mu, md = oracle.unitarity(U)
    assert mu < 1e-13 and md < 1e-13


# --------------------------------------------------------------------------
# P-14  results do not depend on the OpenMP thread count (bitwise)
# --------------------------------------------------------------------------
_THREAD_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import synth, oracle
U = synth.random_links((8, 8, 4, 4), 15)
U2, tf, tt, _ = oracle.step((8, 8, 4, 4), U, 5)
sys.stdout.write(np.concatenate([tf, tt, U2.view(np.float64).ravel()[:5000]]).tobytes().hex())
"""


def test_thread_count_independence(oracle_lib):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for n in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=n)
        r = subprocess.run([sys.executable, "-c", _THREAD_SCRIPT.format(root=root)],
                           env=env, capture_output=True, text=True, check=True)
        outs.append(r.stdout)
    assert outs[0] == outs[1]


# --------------------------------------------------------------------------
# stored trajectory (written by tests/golden/make_golden.py from the oracle)
# --------------------------------------------------------------------------
def test_golden_trajectory_8x4_seed1(oracle_lib):
    path = os.path.join(os.path.dirname(__file__), "golden", "traj_8x8x8x8_seed1.txt")
    rows = np.loadtxt(path)
    dims = (8, 8, 8, 8)
    _, tf, tt, _ = oracle.step(dims, synth.random_links(dims, 1), len(rows) - 1)
    assert np.max(np.abs(tf - rows[:, 1])) <= 1e-13
    assert np.max(np.abs(tt - rows[:, 2]) / rows[:, 2]) <= 1e-10


def _np_unitarity(m):
    """max |M M^dag - 1| (entry-wise complex modulus) and max |det M - 1|, in numpy."""
    m = np.asarray(m, dtype=np.complex128).reshape(-1, 3, 3)
    dev = np.abs(m @ dag(m) - np.eye(3))
    return float(np.max(dev)), float(np.max(np.abs(np.linalg.det(m) - 1.0)))


def test_unitarity_reports_a_perturbed_entry(oracle_lib):
    """The checker must report, not only pass: one entry of one matrix in a
    batch of SU(3) matrices moved by 1e-9 gives that size of error, equal to
    numpy's to rounding."""
    m = synth.haar_su3(5, 50)
    assert max(oracle.unitarity(m)) <= 1e-14
    for k, (i, j) in ((0, (0, 0)), (23, (1, 2)), (49, (2, 1))):
        p = m.copy()
        p[k, i, j] += 1e-9 * (1 + 1j)
        mu, md = oracle.unitarity(p)
        nu, nd = _np_unitarity(p)
        assert 5e-10 <= mu <= 5e-9 and 1e-10 <= md <= 5e-9
        assert abs(mu - nu) <= 1e-15 and abs(md - nd) <= 1e-15


def test_unitarity_reports_a_u3_phase(oracle_lib):
    """A U(3) matrix with det = exp(i phi) is unitary but not special: the
    unitarity error stays at rounding and the det error is |exp(i phi) - 1|."""
    m = synth.haar_su3(6, 8)
    for phi in (1e-6, 0.3, np.pi / 2, 3.0):
        p = m.copy()
        p[3] = p[3] * np.exp(1j * phi / 3.0)
        mu, md = oracle.unitarity(p)
        assert mu <= 1e-14
        assert abs(md - 2.0 * np.sin(phi / 2.0)) <= 1e-15 * max(1.0, 1e3 * phi)
        nu, nd = _np_unitarity(p)
        assert abs(mu - nu) <= 1e-15 and abs(md - nd) <= 1e-15


def test_unitarity_reports_nonfinite(oracle_lib):
    """A NaN anywhere in the batch makes both reported errors NaN (a checker
    that skipped it would pass a broken field)."""
    m = synth.haar_su3(7, 10)
    for k in (0, 4, 9):
        p = m.copy()
        p[k, 1, 1] = complex(np.nan, 0.0)
        mu, md = oracle.unitarity(p)
        assert np.isnan(mu) and np.isnan(md)


def _rand_su3_algebra(rng, n, scale):
    """n random anti-Hermitian traceless 3x3 matrices with Frobenius norm ~ scale."""
    a = rng.normal(size=(n, 3, 3)) + 1j * rng.normal(size=(n, 3, 3))
    x = a - dag(a)
    x -= np.trace(x, axis1=1, axis2=2)[:, None, None] * np.eye(3) / 3.0
    return x * (scale / np.linalg.norm(x, axis=(1, 2)))[:, None, None]


def test_expm_matches_scipy_and_eigendecomposition(oracle_lib):
    """The oracle's matrix exponential (eq. gx evaluated exactly) against
    scipy.linalg.expm on general complex matrices and against the spectral
    formula V diag(exp(i l)) V^dag for anti-Hermitian X = i V diag(l) V^dag."""
    rng = np.random.default_rng(31)
    general = (rng.normal(size=(40, 3, 3)) + 1j * rng.normal(size=(40, 3, 3))) * \
        np.logspace(-9, 0.7, 40)[:, None, None]
    ours = oracle.expm(general)
    for m, e in zip(general, ours):
        ref = scipy.linalg.expm(m)
        assert np.max(np.abs(e - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    for scale in (1e-9, 1e-3, 0.3, 2.0, 6.0):
        x = _rand_su3_algebra(rng, 20, scale)
        e = oracle.expm(x)
        lam, v = np.linalg.eigh(-1j * x)
        ref = (v * np.exp(1j * lam)[:, None, :]) @ dag(v)
        assert np.max(np.abs(e - ref)) <= 2e-14 * max(1.0, scale)
        mu, md = oracle.unitarity(e)
        assert mu <= 1e-13 and md <= 1e-13
    d = np.diag([0.3j, -1.1j, 0.8j])
    assert np.max(np.abs(oracle.expm(d[None])[0] - np.diag(np.exp(np.diag(d))))) <= 1e-15


def test_exact_exponential_update(oracle_lib):
    """The update with g = exp(alpha/2 dtilde): g equals expm of the filtered
    field, the plaquette is unchanged, F rises, the linear-regime contraction
    (1 - alpha p2max)^2 is the same as the first-order update's, and a
    generator field converges."""
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 17)
    o = oracle.opts(expo=True)
    _, _, delta = oracle.measure(dims, U)
    dt = oracle.filter_delta(dims, delta, o)
    g = oracle.gauge(dims, dt, ALPHA, expo=True)
    ref = np.array([scipy.linalg.expm(0.5 * ALPHA * m) for m in dt.reshape(-1, 3, 3)]).reshape(g.shape)
    assert np.max(np.abs(g - ref)) <= 1e-13
    mu, md = oracle.unitarity(g)
    assert mu <= 1e-13 and md <= 1e-13
    U1, tf, _, _ = oracle.step(dims, U, 6, o)
    assert abs(oracle.plaquette(dims, U1) - oracle.plaquette(dims, U)) <= 1e-12
    assert np.all(np.diff(tf) >= -1e-14)
    Us = synth.small_field(dims, 5, eps=1e-5)
    _, _, th, _ = oracle.step(dims, Us, 1, o)
    assert abs(th[1] / th[0] / (1 - ALPHA * 16) ** 2 - 1) <= 1e-4
    _, it, _, th_end, conv, _ = oracle.fix(dims, U, o)
    assert conv and th_end < 1e-15 and it < 200
