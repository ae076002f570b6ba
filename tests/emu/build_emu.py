"""Build the library's HIP sources for the CPU against tests/emu/include.

TEST INFRASTRUCTURE: produces tests/emu/liblgf_emu.so (and, with --asan, an
AddressSanitizer-instrumented copy) so index arithmetic and bounds of the
kernels and the runtime can be exercised without a GPU.
"""
import fcntl
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRCS = [os.path.join(ROOT, "paper_1206_0675_amd", "csrc", f) for f in ("lgf.hip", "batch.hip", "mlp.hip", "noalloc.hip", "wilson.hip", "fft_study.hip")]


def _inputs():
    pats = [os.path.join(ROOT, "paper_1206_0675_amd", "csrc", "*"), os.path.join(ROOT, "include", "*"),
            os.path.join(HERE, "include", "*", "*"), os.path.join(HERE, "include", "*"), os.path.abspath(__file__)]
    return [f for p in pats for f in glob.glob(p) if os.path.isfile(f)]


def build(asan: bool = False) -> str:
    """Compile unless the library is newer than every source and header.  A
    lock file serialises concurrent test processes."""
    out = os.path.join(HERE, "liblgf_emu_asan.so" if asan else "liblgf_emu.so")
    with open(out + ".lock", "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        if os.path.exists(out) and os.path.getmtime(out) > max(os.path.getmtime(f) for f in _inputs()):
            return out
        tmp = f"{out}.{os.getpid()}.tmp"
        cmd = ["g++", "-std=gnu++20", "-x", "c++", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-mfma",
               "-ffp-contract=off", "-I" + os.path.join(HERE, "include"), "-I" + os.path.join(ROOT, "include"),
               "-I" + os.path.join(ROOT, "paper_1206_0675_amd", "csrc")] + SRCS + ["-o", tmp]
        if asan:
            cmd[5:5] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(asan="--asan" in sys.argv))
