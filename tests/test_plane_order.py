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


ZT_SRC = r"""
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#include "runtime.hpp"
template <typename T>
int check(const int* dims, int tb, int& launches)
{
    const lgf::Geo g = lgf::rt::make_geo<T>(dims, tb);
    const int l = lgf::rt::zt_part_log<T>(g);
    const int nchunk = (g.NP >> g.logW) * 4, lnh = g.logW - l;
    const int blocks = lgf::rt::zt_blocks(g, l);
    int bad = (blocks != (nchunk << lnh)) + (lgf::rt::zt_lds<T>(g, l) > lgf::rt::kMaxLdsZt) + (l < 0 || l > g.logW);
    std::vector<int> seen((size_t)nchunk << lnh, 0);
    for (int b = 0; b < blocks; ++b) {
        int h, chunk;
        lgf::zt_part_of_block(b, nchunk, lnh, h, chunk);
        if (chunk < 0 || chunk >= nchunk || h < 0 || h >= (1 << lnh)) { ++bad; continue; }
        ++seen[((size_t)chunk << lnh) + h];
    }
    for (int v : seen) bad += v != 1;
    ++launches;
    return bad;
}
int main()
{
    int bad = 0, launches = 0;
    for (int lx = 4; lx <= 128; lx *= 2)
        for (int ly = 4; ly <= 128; ly *= 2)
            for (int lz = 4; lz <= 128; lz *= 2)
                for (int lt = 4; lt <= 128; lt *= 2) {
                    const int d[4] = {lx, ly, lz, lt};
                    for (int tb : {32, 64, 128}) {
                        if (lgf::rt::shape_fits<double>(d, 64)) bad += check<double>(d, tb, launches);
                        if (lgf::rt::shape_fits<float>(d, 64)) bad += check<float>(d, tb, launches);
                    }
                }
    std::printf("%d %d\n", launches, bad);
    return bad != 0;
}
"""


def test_zt_part_map_covers_every_chunk_once(tmp_path):
    """Every (tile, field) chunk and part of the (z, t) launch is handled by
    exactly one block, its LDS fits, for every supported shape, both
    precisions and every tile width the autotuner may choose."""
    src = tmp_path / "zt.cpp"
    exe = tmp_path / "zt"
    src.write_text(ZT_SRC)
    inc = ["-I" + os.path.join(HERE, "emu", "include"), "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1206_0675_amd", "csrc")]
    r = subprocess.run(["g++", "-std=gnu++20", "-O1", "-pthread", *inc, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr[-2000:])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    launches, bad = (int(v) for v in out.stdout.split())
    assert out.returncode == 0 and bad == 0 and launches > 1000
