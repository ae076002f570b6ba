"""The C ABI on a machine without a GPU: the gfx950 library loads, exports
every function include/*.h declares, and its host-only paths (defaults,
validation, argument checks before any device call, error strings) behave
as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from paper_1206_0675_amd import lgf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lgf.DEFAULT_LIB):
        from paper_1206_0675_amd import build
        build.build()
    return lgf.load_library()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lgf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lgf_create", "lgf_destroy", "lgf_load_links", "lgf_store_links", "lgf_step", "lgf_fix",
                     "lgf_measure", "lgf_validate_links", "lgf_default_params", "lgf_wilson_create",
                     "lgf_wilson_update", "lgf_wilson_store", "lgf_wilson_plaquette"]:
        assert required in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_header(L, tmp_path):
    """ctypes mirrors of lgf_params / lgf_stats agree with the C compiler's layout."""
    src = tmp_path / "layout.c"
    fields = {"lgf_params": lgf.Params, "lgf_stats": lgf.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lgf.h"', 'int main(void) {']
    for cname, cls in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in fields.items():
        assert int(got[cname]) == C.sizeof(cls)
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_default_params(L):
    p = lgf.default_params((8, 8, 8, 8), L)
    assert p.alpha == 0.08 and p.theta_stop == 1e-15 and p.theta_switch == 1e-6
    assert p.precision == lgf.FP64 and p.storage == lgf.STORE18 and p.accel == lgf.ACCEL_FOURIER
    assert p.max_iter == 100000 and p.poll_every == 16 and p.unit_tol == 1e-12
    assert L.lgf_default_params(None) == lgf.E_INVALID_ARG


def test_validate_links_host_only(L):
    dims = (4, 4, 4, 2)
    U = synth.random_links(dims, 1)
    assert lgf.validate_links(dims, U, lib=L) == (lgf.OK, -1)
    bad = U.copy()
    bad[1, 2, 3, 0, 2] *= 1.0 + 1e-9                 # site (x=0,y=3,z=2,t=1), mu=2
    rc, first = lgf.validate_links(dims, bad, lib=L)
    s = ((1 * 4 + 2) * 4 + 3) * 4 + 0
    assert rc == lgf.E_NOT_UNITARY and first == s * 4 + 2
    nan = U.copy()
    nan[0, 0, 0, 1, 3, 1, 1] = np.nan
    assert lgf.validate_links(dims, nan, lib=L) == (lgf.E_NONFINITE, 1 * 4 + 3)
    assert lgf.validate_links(dims, bad, tol=1e-6, lib=L)[0] == lgf.OK


@pytest.mark.parametrize("dims, code", [((6, 8, 8, 8), lgf.E_UNSUPPORTED_SHAPE), ((2, 8, 8, 8), lgf.E_UNSUPPORTED_SHAPE),
                                        ((8, 8, 8, 256), lgf.E_UNSUPPORTED_SHAPE),
                                        ((128, 128, 8, 8), lgf.E_UNSUPPORTED_SHAPE),
                                        ((8, 8, 128, 128), lgf.E_UNSUPPORTED_SHAPE)])
def test_create_rejects_shapes_before_touching_the_device(L, dims, code):
    with pytest.raises(lgf.LgfError) as e:
        lgf.Context(dims, lib=L)
    assert e.value.code == code


@pytest.mark.parametrize("field, value", [("precision", 7), ("storage", 10), ("step", 3), ("accel", 2),
                                          ("alpha", 0.0), ("alpha", float("nan")), ("theta_stop", -1.0),
                                          ("max_iter", -1), ("poll_every", 0)])
def test_create_rejects_params_before_touching_the_device(L, field, value):
    with pytest.raises(lgf.LgfError) as e:
        lgf.Context((8, 8, 8, 8), lib=L, **{field: value})
    assert e.value.code == lgf.E_INVALID_ARG


@pytest.mark.parametrize("precision", [lgf.FP32, lgf.MIXED])
def test_learned_step_needs_fp64(L, precision):
    with pytest.raises(lgf.LgfError) as e:
        lgf.Context((8, 8, 8, 8), lib=L, step=lgf.STEP_LEARNED, precision=precision)
    assert e.value.code == lgf.E_INVALID_ARG


def test_error_strings(L):
    for code in range(0, -10, -1):
        assert L.lgf_strerror(code) != b"unknown status"
    assert L.lgf_strerror(-100) == b"unknown status"
    assert L.lgf_destroy(None) == lgf.OK
    assert L.lgf_kernel_name(0) == b"load" and L.lgf_kernel_name(99) is None


def test_malformed_model_rejected_before_touching_the_device(L):
    import numpy as np
    n = L.lgf_model_bytes()
    good_size = bytes(n)                                  # right size, zero header
    for blob in (good_size, bytes(n - 2), b""):
        with pytest.raises(lgf.LgfError) as e:
            lgf.mlp_eval(blob, np.zeros((2, 16)), lib=L)
        assert e.value.code == lgf.E_MODEL


def test_product_path_has_no_fallback(tmp_path):
    with pytest.raises(ImportError):
        lgf.load_library(str(tmp_path / "missing.so"))


def test_wilson_generator_argument_checks_before_device_calls(L):
    h = C.c_void_p()
    for dims, beta, code in (((3, 4, 4, 4), 6.0, lgf.E_UNSUPPORTED_SHAPE), ((4, 4, 4, 2048), 6.0, lgf.E_UNSUPPORTED_SHAPE),
                             ((4, 4, 4, 4), -0.5, lgf.E_INVALID_ARG), ((4, 4, 4, 4), float("nan"), lgf.E_INVALID_ARG)):
        d = (C.c_int32 * 4)(*dims)
        assert L.lgf_wilson_create(d, beta, 1, C.byref(h)) == code
        assert L.lgf_wilson_last_error(None)
    assert L.lgf_wilson_create(None, 6.0, 1, C.byref(h)) == lgf.E_INVALID_ARG
    assert L.lgf_wilson_destroy(None) == lgf.E_INVALID_ARG
    assert L.lgf_wilson_device_links(None) is None
