"""GPU parity of the 4D-FFT decomposition study (include/lgf_study.h): each
decomposition (also the one whose t-axis DFTs run on the matrix cores)
applies the oracle's filter F^-1 (p2max/p^2) F / V to the
packed Delta fields, to 1e-13 of the largest output at small shapes; at 32^4
(the benchmark's shape) the three agree with one another to the same bound."""
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_1206_0675_amd import lgf

pytestmark = pytest.mark.gpu

VARIANTS = (lgf.FFT_1DX4, lgf.FFT_2D1D1D, lgf.FFT_2D2D, lgf.FFT_2D1D1D_MFMA)


@pytest.fixture(scope="module")
def L():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lgf.load_library()


def announce(msg):
    print(f"\n[gpu] {msg}", flush=True)
    sys.stdout.flush()


def pack(D):
    return np.ascontiguousarray(np.stack([D[..., 0, 1], D[..., 0, 2], D[..., 1, 2],
                                          D[..., 0, 0].imag + 1j * D[..., 1, 1].imag]))


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (16, 8, 4, 32), (4, 16, 32, 8), (16, 16, 16, 16), (8, 4, 4, 64)])
def test_decompositions_match_oracle(L, dims):
    announce(f"fft study dims={dims}")
    U = synth.random_links(dims, 4)
    _, _, delta = oracle.measure(dims, U)
    ref = pack(oracle.filter_delta(dims, delta))
    f = pack(delta)
    for v in VARIANTS:
        if v == lgf.FFT_2D1D1D_MFMA and dims[3] < 16:
            continue
        out, _ = lgf.fft_study(dims, v, f, lib=L)
        assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref)), v


def test_decompositions_agree_at_full_size(L):
    import torch
    dims = (32, 32, 32, 32)
    announce("fft study 32^4 on device buffers")
    g = torch.Generator(device="cpu").manual_seed(5)
    f = torch.complex(torch.randn((4, 32, 32, 32, 32), dtype=torch.float64, generator=g),
                      torch.randn((4, 32, 32, 32, 32), dtype=torch.float64, generator=g)).cuda()
    outs = []
    for v in VARIANTS:
        out, ms = lgf.fft_study(dims, v, f, reps=2, lib=L)
        torch.cuda.synchronize()
        assert ms > 0.0
        outs.append(out.cpu().numpy())
    scale = np.max(np.abs(outs[2]))
    for i in (0, 1, 3):
        assert np.max(np.abs(outs[i] - outs[2])) <= 1e-13 * scale, i
