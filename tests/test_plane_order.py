"""The block -> plane order of the per-plane kernels is a permutation.

plane_of_block (kernels.hpp) deals the (z, t) planes to blocks in an
XCD-aware order; every plane must be handled exactly once, for every
supported shape.  The header is compiled for the host (g++, against the
CPU emulation header) and checked exhaustively.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SRC = r"""
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#include "kernels.hpp"
int main()
{
    int bad = 0, shapes = 0;
    for (int Lz = 4; Lz <= 128; Lz *= 2)
        for (int Lt = 4; Lt <= 128; Lt *= 2) {
            lgf::Geo g{};
            g.L[0] = g.L[1] = 4;
            g.L[2] = Lz;
            g.L[3] = Lt;
            g.NQ = Lz * Lt;
            std::vector<int> seen(g.NQ, 0);
            for (int b = 0; b < g.NQ; ++b) {
                const int q = lgf::plane_of_block(b, g);
                if (q < 0 || q >= g.NQ) { ++bad; continue; }
                ++seen[q];
            }
            for (int q = 0; q < g.NQ; ++q) bad += seen[q] != 1;
            ++shapes;
        }
    std::printf("%d %d\n", shapes, bad);
    return bad != 0;
}
"""


def test_plane_order_is_a_permutation(tmp_path):
    src = tmp_path / "order.cpp"
    exe = tmp_path / "order"
    src.write_text(SRC)
    inc = ["-I" + os.path.join(HERE, "emu", "include"), "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1206_0675_amd", "csrc")]
    r = subprocess.run(["g++", "-std=gnu++20", "-O1", "-pthread", *inc, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr[-2000:])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    shapes, bad = (int(v) for v in out.stdout.split())
    assert out.returncode == 0 and bad == 0 and shapes == 36
