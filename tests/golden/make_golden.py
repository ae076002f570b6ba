"""Write the stored oracle trajectories under tests/golden/.

Calls only the FP64 oracle and the seeded generator.  Rerun after a change
to the oracle's arithmetic and name the passage of the paper that justifies
that change in the commit.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    dims = (8, 8, 8, 8)
    U = synth.random_links(dims, 1)
    _, it, _, _, _, _ = oracle.fix(dims, U)
    _, tf, tt, _ = oracle.step(dims, U, it)
    path = os.path.join(HERE, "traj_8x8x8x8_seed1.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, 8^4, synth.random_links seed 1 (eps for plaquette 0.6),\n")
        f.write("# alpha 0.08, Fourier acceleration p2max/p2; stop theta < 1e-15 (Section 2).\n")
        f.write(f"# {it} gauge transformations to convergence.  columns: iteration F theta\n")
        for k in range(it + 1):
            f.write(f"{k:3d} {tf[k]:.17e} {tt[k]:.17e}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
