"""Compile the HIP library for gfx950 into paper_1206_0675_amd/liblgf.so.

    python -m paper_1206_0675_amd.build        (or python paper_1206_0675_amd/build.py)

Packed FP32 instructions are disabled (-packed-fp32-ops) on purpose.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblgf.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("lgf.hip", "batch.hip", "mlp.hip", "noalloc.hip", "wilson.hip", "fft_study.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC] + flags() + list(extra) + SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
