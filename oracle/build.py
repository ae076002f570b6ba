"""Build the FP64 CPU oracle (test infrastructure) as oracle/liblgfo.so with gcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblgfo.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp", "-fcx-limited-range",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-ffp-contract=off", os.path.join(HERE, "lgfo.c"), os.path.join(HERE, "wilson.c"),
           "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
