"""Build the library's HIP sources for the CPU against tests/emu/include.

TEST INFRASTRUCTURE: produces tests/emu/liblgf_emu.so (and, with --asan, an
AddressSanitizer-instrumented copy) so index arithmetic and bounds of the
kernels and the runtime can be exercised without a GPU.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRCS = [os.path.join(ROOT, "paper_1206_0675_amd", "csrc", f) for f in ("lgf.hip", "batch.hip", "mlp.hip")]


def build(asan: bool = False) -> str:
    out = os.path.join(HERE, "liblgf_emu_asan.so" if asan else "liblgf_emu.so")
    cmd = ["g++", "-std=gnu++20", "-x", "c++", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-mfma", "-ffp-contract=off",
           "-I" + os.path.join(HERE, "include"), "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1206_0675_amd", "csrc")] + SRCS + ["-o", out + ".tmp"]
    if asan:
        cmd[5:5] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(asan="--asan" in sys.argv))
