"""The allocation-free entry point lgf_fix_noalloc against the context path
(lgf_create, lgf_load_links, lgf_fix, lgf_store_links) on the GPU: two calls
in a row on device-resident links, the second on a smaller lattice, must give
the same links, F, theta and iteration count.  Also its host-side refusals."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from paper_1206_0675_amd import lgf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    return lgf.load_library()


def context_fix(L, dims, U, storage):
    with lgf.Context(dims, lib=L, storage=storage) as ctx:
        ctx.load(U)
        st = ctx.fix()
        return ctx.store(), st


@pytest.mark.parametrize("storage", [12, 18])
def test_noalloc_matches_context_path_twice(L, storage):
    import torch
    cases = [((16, 16, 8, 16), 31), ((8, 8, 8, 8), 32)]      # second call: smaller lattice
    for dims, seed in cases:
        print(f"noalloc vs context: dims {dims} seed {seed} storage {storage}", flush=True)
        U = synth.random_links(dims, seed)
        Uin = torch.from_numpy(U.view(np.float64).copy()).cuda()
        Uout = torch.full_like(Uin, float("nan"))
        st, rc = lgf.fix_noalloc(Uin, Uout, lib=L, storage=storage)
        torch.cuda.synchronize()
        assert rc == lgf.OK, L.lgf_last_error(None).decode()
        Uc, sc = context_fix(L, dims, U, storage)
        Un = Uout.cpu().numpy().view(np.complex128).reshape(U.shape)
        # same kernels, launch shape and order: the same bits
        assert np.array_equal(Un, Uc)
        assert st.iter == sc.iter and st.F == sc.F and st.theta == sc.theta and st.theta < 1e-15
        # and against the FP64 oracle to the full-run bar
        _, it_o, Fo, _, conv, _ = oracle.fix(dims, U, oracle.opts(store12=(storage == 12)))
        assert conv and abs(st.F - Fo) <= 1e-9 and abs(st.iter - it_o) <= 1
        assert np.array_equal(Uin.cpu().numpy(), U.view(np.float64))      # input untouched


def test_noalloc_in_place_and_refusals(L):
    import torch
    dims = (8, 8, 4, 8)
    U = synth.random_links(dims, 33)
    buf = torch.from_numpy(U.view(np.float64).copy()).cuda()
    st, rc = lgf.fix_noalloc(buf, buf, lib=L, storage=12)
    assert rc == lgf.OK
    Uc, sc = context_fix(L, dims, U, 12)
    assert np.array_equal(buf.cpu().numpy().view(np.complex128).reshape(U.shape), Uc) and st.iter == sc.iter
    # refused before any device work: too large for the static scratch, or not FP64
    big = torch.empty(1, device="cuda", dtype=torch.float64)
    p = lgf.default_params((32, 32, 32, 32), L)
    assert L.lgf_fix_noalloc(C.byref(p), C.c_void_p(big.data_ptr()), C.c_void_p(big.data_ptr()), None) \
        == lgf.E_UNSUPPORTED_SHAPE
    assert b"scratch" in L.lgf_last_error(None)
    p = lgf.default_params(dims, L, precision=lgf.MIXED)
    assert L.lgf_fix_noalloc(C.byref(p), C.c_void_p(big.data_ptr()), C.c_void_p(big.data_ptr()), None) \
        == lgf.E_INVALID_ARG
