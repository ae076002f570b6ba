"""GPU parity of the Wilson-action generator (include/lgf_wilson.h) against
the reference in oracle/wilson.c, through the C ABI.

Links after heatbath and overrelaxation sweeps agree with the reference to
1e-12 (the two sides draw the same Philox numbers and take their sampler
decisions in FP64; only the last bits of log, cos, sin and exp may differ),
at small shapes and at 32^4 for a full sweep; overrelaxation keeps the
plaquette; the generated fields feed the gauge-fixing context directly.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import wilson as owil
from paper_1206_0675_amd import lgf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lgf.load_library()


def announce(msg):
    print(f"\n[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dims, beta, start", [((4, 4, 4, 4), 5.9, "random"), ((8, 4, 6, 2), 6.2, "cold"),
                                               ((4, 8, 4, 8), 0.4, "cold")])
def test_sweeps_match_oracle(L, dims, beta, start):
    """Sweep by sweep from the same input links: the heatbath is chaotic, so
    the last-bit differences of the math functions grow over many sweeps;
    each sweep is compared on its own."""
    announce(f"wilson sweeps dims={dims} beta={beta} start={start}")
    U = synth.random_links(dims, 3) if start == "random" else owil.cold(dims)
    with lgf.WilsonGenerator(dims, beta, 77, lib=L) as g:
        g.load(U)
        prev, n = U, 0
        for kind in (lgf.HEATBATH, lgf.OVERRELAX, lgf.HEATBATH, lgf.OVERRELAX, lgf.OVERRELAX, lgf.HEATBATH):
            g.sweep(kind)
            Uo, sk = owil.sweep(dims, prev, beta, 77, n, kind)
            Ug = g.store()
            assert np.max(np.abs(Ug - Uo)) <= 1e-12 and sk == 0, (kind, n)
            assert max(oracle.unitarity(Ug)) <= 1e-13
            prev, n = Ug, n + (kind == lgf.HEATBATH)
        assert g.skipped() == 0 and g.sweep_index == n == 3


def test_update_is_its_sweeps(L):
    dims = (4, 4, 4, 8)
    announce("wilson update = its sweeps")
    U = synth.random_links(dims, 4)
    with lgf.WilsonGenerator(dims, 5.8, 8, lib=L) as a, lgf.WilsonGenerator(dims, 5.8, 8, lib=L) as b:
        a.load(U)
        b.load(U)
        a.update(2, 2)
        for kind in (lgf.HEATBATH, lgf.OVERRELAX, lgf.OVERRELAX) * 2:
            b.sweep(kind)
        assert np.array_equal(a.store(), b.store()) and a.sweep_index == b.sweep_index == 2


def test_plaquette_and_determinism(L):
    dims = (8, 8, 8, 8)
    announce("wilson plaquette and determinism 8^4")
    with lgf.WilsonGenerator(dims, 6.0, 5, lib=L) as a, lgf.WilsonGenerator(dims, 6.0, 5, lib=L) as b:
        a.update(5, 2)
        b.update(5, 2)
        Ua, Ub = a.store(), b.store()
        assert np.array_equal(Ua, Ub)
        assert abs(a.plaquette() - oracle.plaquette(dims, Ua)) <= 1e-13
        b.sweep_index = 0
        b.cold()
        assert np.array_equal(b.store(), owil.cold(dims))


def test_full_size_sweep_matches_oracle(L):
    """One heatbath and one overrelaxation sweep at 32^4 (the benchmark's
    shape), every link against the reference; overrelaxation keeps the
    plaquette."""
    dims = (32, 32, 32, 32)
    announce("wilson full-size sweep 32^4")
    U = synth.random_links(dims, 9, workers=8)
    with lgf.WilsonGenerator(dims, 6.0, 123, lib=L) as g:
        g.load(U)
        g.sweep(lgf.HEATBATH)
        Ug = g.store()
        Uo, sk = owil.sweep(dims, U, 6.0, 123, 0, owil.HEATBATH)
        assert np.max(np.abs(Ug - Uo)) <= 1e-12 and g.skipped() == sk == 0
        p0 = g.plaquette()
        g.sweep(lgf.OVERRELAX)
        assert abs(g.plaquette() - p0) <= 1e-12
        assert abs(p0 - oracle.plaquette(dims, Ug)) <= 1e-13


def test_generated_field_is_gauge_fixed(L):
    """A thermalised beta = 6.0 field at 16^4 goes to the gauge-fixing
    context on the device and converges; it needs far more iterations than
    the synthetic fields, and fixing leaves the plaquette unchanged."""
    dims = (16, 16, 16, 16)
    announce("wilson field gauge-fixed 16^4")
    with lgf.WilsonGenerator(dims, 6.0, 31, lib=L) as g:
        g.update(60, 4)
        P = g.plaquette()
        assert 0.58 < P < 0.61          # the beta = 6.0 plaquette is about 0.594
        with lgf.Context(dims, lib=L, max_iter=20000) as c:
            c.load_device(g.device_links)
            st = c.fix()
            Uf = c.store()
    assert st.theta < 1e-15 and st.iter > 200
    assert abs(oracle.plaquette(dims, Uf) - P) <= 1e-12
    assert oracle.measure(dims, Uf)[1] < 1e-15


def test_hand_off_of_loaded_and_swept_links(L):
    """The sweeps keep rows 0 and 1 of each link and rebuild row 2; the
    canonical copy behind store and the device hand-off holds the loaded
    links unchanged until a sweep, then the swept ones."""
    dims = (4, 4, 4, 8)
    announce("wilson hand-off of loaded and swept links")
    U = synth.random_links(dims, 6)
    with lgf.WilsonGenerator(dims, 6.0, 3, lib=L) as g:
        g.load(U)
        assert np.array_equal(g.store(), U)
        with lgf.Context(dims, lib=L, storage=18) as c:
            c.load_device(g.device_links)
            assert np.max(np.abs(c.store() - U)) <= 1e-15
        g.sweep(lgf.OVERRELAX)
        Ug = g.store()
        Uo, _ = owil.sweep(dims, U, 6.0, 3, 0, owil.OVERRELAX)
        assert np.max(np.abs(Ug - Uo)) <= 1e-12
        with lgf.Context(dims, lib=L, storage=18) as c:
            c.load_device(g.device_links)
            assert np.max(np.abs(c.store() - Ug)) <= 1e-15
