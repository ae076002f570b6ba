"""FP64 CPU oracle for Fourier-accelerated Landau gauge fixing.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke test
and the CPU-baseline leg of the benchmark; never by the GPU library.
"""
from .lgfo import *  # noqa: F401,F403
