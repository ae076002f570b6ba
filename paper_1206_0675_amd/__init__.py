"""MI355X (gfx950) Landau gauge fixing by Fourier-accelerated steepest descent.

The iteration runs in hand-written HIP kernels behind the C ABI of
include/lgf.h (library liblgf.so); `lgf` is its ctypes binding.
"""
from . import lgf  # noqa: F401
from .lgf import Context, LgfError, default_params, load_library, validate_links  # noqa: F401
