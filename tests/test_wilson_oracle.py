"""Pins of the Wilson-action generator reference (oracle/wilson.c).

Each test checks the reference against something other than itself: an
independent Philox implementation (numpy's), moments of the x0 density by
quadrature, the plaquette sum (an identity the staple must satisfy), gauge
covariance of the staple and gauge invariance of the action, the exact
action conservation of overrelaxation, and the
strong-coupling limit <P> = beta/18 + O(beta^2) of the Wilson action.  A
wrong staple index or dagger, a wrong subgroup projection, a wrong constant
in the sampler or a broken counter fails at least one of them.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
import synth
from oracle import wilson as W


def test_philox_matches_numpy():
    """numpy's Philox is Philox4x64-10; it increments its counter before
    each block, so its first block is ours at counter + 1."""
    rng = np.random.default_rng(5)
    cases = [((1, 0, 0, 0), (0, 0)), ((2, 3, 4, 5), (6, 7)), ((2**64 - 1, 5, 0, 2**63), (2**64 - 1, 1))]
    cases += [(tuple(int(v) for v in rng.integers(1, 2**63, 4)), tuple(int(v) for v in rng.integers(0, 2**63, 2)))
              for _ in range(5)]
    for ctr, key in cases:
        before = list(ctr)
        before[0] -= 1
        bg = np.random.Philox(counter=np.array(before, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
        assert W.philox4x64(ctr, key) == [int(v) for v in bg.random_raw(4)], (ctr, key)


@pytest.mark.parametrize("c", [0.0, 0.3, 0.999, 1.0, 3.0, 25.0])
def test_x0_sampler_moments(c):
    """Mean and mean square of x0 against the density sqrt(1-x^2) exp(c x)
    integrated numerically (both sampler branches: c < 1 and c >= 1)."""
    n = 200000
    x, failed = W.x0_sample(c, 3, n)
    assert failed == 0 and np.all(np.abs(x) <= 1.0)
    w = lambda t, k: t ** k * np.sqrt(1 - t * t) * np.exp(c * (t - 1))   # noqa: E731
    z = quad(w, -1, 1, args=(0,))[0]
    m1, m2, m4 = (quad(w, -1, 1, args=(k,))[0] / z for k in (1, 2, 4))
    assert abs(x.mean() - m1) <= 5 * np.sqrt((m2 - m1 ** 2) / n)
    assert abs((x * x).mean() - m2) <= 5 * np.sqrt((m4 - m2 ** 2) / n)


def test_staple_sum_is_four_plaquette_sums(oracle_lib):
    """Every plaquette holds four links, so the sum over links of
    Re Tr(U A) is 4 * 18 V <P> (the plaquette written independently in
    lgfo.c)."""
    for dims in ((4, 4, 4, 4), (4, 8, 2, 4)):
        U = synth.random_links(dims, 12)
        V = int(np.prod(dims))
        s = W.link_action_sum(dims, U)
        assert abs(s - 72 * V * oracle.plaquette(dims, U)) <= 1e-12 * 72 * V


def test_staple_gauge_covariance_and_action_invariance(oracle_lib):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag takes A_mu(x) to g(x+mu) A_mu(x) g(x)^dag
    and leaves the action unchanged."""
    dims = (4, 4, 2, 8)
    U = synth.random_links(dims, 13)
    lx, ly, lz, lt = dims
    g = synth.haar_su3(14, lx * ly * lz * lt).reshape(lt, lz, ly, lx, 3, 3)
    Ug = oracle.transform(dims, U, g)
    gf = g.reshape(-1, 3, 3)
    rng = np.random.default_rng(3)
    for site in rng.integers(0, lx * ly * lz * lt, 6):
        for mu in range(4):
            c = np.unravel_index(int(site), (lt, lz, ly, lx))[::-1]
            c = list(c)
            c[mu] = (c[mu] + 1) % dims[mu]
            xm = ((c[3] * lz + c[2]) * ly + c[1]) * lx + c[0]
            A, Ag = W.staple(dims, U, site, mu), W.staple(dims, Ug, site, mu)
            assert np.max(np.abs(Ag - gf[xm] @ A @ gf[site].conj().T)) <= 1e-12
    assert abs(W.link_action_sum(dims, Ug) - W.link_action_sum(dims, U)) <= 1e-11


def test_overrelaxation_conserves_action(oracle_lib):
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 15)
    U1, _ = W.sweep(dims, U, 6.0, 1, 0, W.OVERRELAX)
    assert np.max(np.abs(U1 - U)) > 1e-2
    P0, P1 = oracle.plaquette(dims, U), oracle.plaquette(dims, U1)
    assert abs(P1 - P0) <= 1e-13
    # one link: Re Tr(U A) with its staple A is kept while U moves
    A = W.staple(dims, U, 37, 2)
    U2, _ = W.link_update(dims, U, 37, 2, 6.0, 1, 0, W.OVERRELAX)
    u0, u1 = U.reshape(-1, 4, 3, 3)[37, 2], U2.reshape(-1, 4, 3, 3)[37, 2]
    assert np.max(np.abs(u1 - u0)) > 1e-2
    assert abs(np.trace(u1 @ A).real - np.trace(u0 @ A).real) <= 1e-13


def test_heatbath_stays_in_su3_and_follows_its_counters(oracle_lib):
    dims = (4, 4, 4, 4)
    U, sk = W.generate(dims, W.cold(dims), 5.7, 21, 0, 3, 1)
    assert sk == 0
    assert max(oracle.unitarity(U)) <= 1e-13
    # the same seed and sweep numbers give the same links; another seed does not
    U2, _ = W.generate(dims, W.cold(dims), 5.7, 21, 0, 3, 1)
    U3, _ = W.generate(dims, W.cold(dims), 5.7, 22, 0, 3, 1)
    assert np.array_equal(U, U2) and np.max(np.abs(U3 - U)) > 1e-2
    # a heatbath sweep numbered n draws from counters (l, n, ...): two sweeps
    # numbered 0, 1 differ from two sweeps numbered 0, 0
    A, _ = W.generate(dims, W.cold(dims), 5.7, 21, 0, 2, 0)
    B, _ = W.sweep(dims, W.sweep(dims, W.cold(dims), 5.7, 21, 0, 0)[0], 5.7, 21, 0, 0)
    assert np.max(np.abs(A - B)) > 1e-2


@pytest.mark.parametrize("beta", [0.0, 0.15, 0.3])
def test_strong_coupling_plaquette(oracle_lib, beta):
    """<P> = <Re Tr U_P / 3> = beta/18 + O(beta^2) for the Wilson action
    (the Haar averages <|Tr U|^2> = 1, <(Tr U)^2> = 0 of SU(3)); 0 at
    beta = 0 (Haar-random links)."""
    dims = (8, 8, 8, 8)
    U, _ = W.generate(dims, W.cold(dims), beta, 11, 0, 10, 1)
    ps = []
    for n in range(30):
        U, sk = W.generate(dims, U, beta, 11, 10 + n, 1, 1)
        assert sk == 0
        ps.append(oracle.plaquette(dims, U))
    ps = np.array(ps)
    err = ps.std() / np.sqrt(len(ps))
    assert abs(ps.mean() - beta / 18) <= 4 * err + beta ** 2 / 100, (ps.mean(), err)
