"""Host-side launch rules of the two-step kernel (k_step_tiled2_api.hpp),
compiled into a small host program and run on the CPU (no GPU call).

Pinned: the default tile heights (9 FP32, 5 FP64 unless their ragged last rows
idle 2 % more sites than one row less) and the default z-chunks: at most 192
planes, and for one launch the longest chunks whose estimated cost,
ceil(blocks / 256) x (planes per chunk + 2) x (a block's time per plane: 1 for the
default height, 8/9 x 1.016 for 8 FP32 rows, 4/5 x 1.085 for 4 FP64 rows), is within
1 % of the least, with the lower height taken when its cost is more than 2 % below
the default height's; against the values worked out by hand below.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = r'''
#include "k_step_tiled2_api.hpp"
#include <cstdio>
int main() {
    const int shapes[][3] = {{512, 512, 512}, {1024, 1024, 1024}, {256, 256, 256},
                             {1024, 1024, 128}, {128, 16, 12}, {64, 8, 8}, {128, 128, 128}};
    for (auto &s : shapes)
        for (int f = 0; f < 2; ++f) {
            int ty = 0, cz = 0, tb = 0, cb = 0;
            ah::tiled2_defaults(f, s[0], s[1], s[2], ty, cz);
            ah::tiled2_defaults(f, s[0], s[1], s[2], tb, cb, false);
            std::printf("%d %d %d %d %d %d %d\n", s[0], s[1], s[2], f, ty, cz, cb);
        }
    int keep_ty = 4, keep_cz = 7;
    ah::tiled2_defaults(false, 512, 512, 512, keep_ty, keep_cz);
    std::printf("keep %d %d\n", keep_ty, keep_cz);
}
'''


@pytest.fixture(scope="module")
def rules(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rules")
    src, exe = d / "rules.cpp", d / "rules"
    src.write_text(PROG)
    subprocess.run([hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1809_00995_amd", "csrc"),
                    "-o", str(exe), str(src)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table, keep = {}, None
    for line in out.splitlines():
        v = line.split()
        if v[0] == "keep":
            keep = (int(v[1]), int(v[2]))
        else:
            nx, ny, nz, f, ty, cz, cb = map(int, v)
            table[(nx, ny, nz, f)] = (ty, cz, cb)
    return table, keep


def test_tile_heights(rules):
    """512^3 FP32: 8-row tiles (512 a plane) cost at best 4 chunks of 128, 8 rounds x 130
    x 0.9031 = 939.2, not 2 % below the 945 of 9 rows: 9.  1024 x 1024 x 128 FP32: 9 rows
    (1824 tiles) cost at best 15 x 66 = 990, 8 rows (2048 tiles, one chunk) 8 x 130 x
    0.9031 = 939.2 < 0.98 x 990: 8.  256^3 FP32: 9 rows (116 tiles, 2 chunks) 1 x 130,
    8 rows (128 tiles) 117.4 < 127.4: 8."""
    table, _ = rules
    assert table[(512, 512, 512, 0)][0] == 9 and table[(512, 512, 512, 1)][0] == 5
    assert table[(1024, 1024, 1024, 0)][0] == 9
    assert table[(1024, 1024, 128, 0)][0] == 8
    assert table[(256, 256, 256, 0)][0] == 8
    # 128 rows: 9-row tiles pad to 135 (5.5 % idle), 8-row tiles none
    assert table[(128, 128, 128, 0)][0] == 8
    # 16 rows in FP64: 5-row tiles pad to 20 (25 %), 4-row tiles none
    assert table[(128, 16, 12, 1)][0] == 4


def test_chunks_for_one_launch(rules):
    """By hand, FP64 512^3 (8 x 103 = 824 tiles a plane): 3 chunks of 171 planes give
    2472 blocks, 10 rounds x 173 = 1730; 4 of 128 give 3296 blocks, 13 x 130 = 1690
    (the least); 5 of 103: 17 x 105 = 1785.  FP32 512^3 (456 tiles): 5 chunks of 103,
    9 rounds x 105 = 945, the least.  1024^3 FP32: 128-plane chunks cost 7410, 171-plane
    7439 (within 1 %, the longer taken)."""
    table, keep = rules
    assert table[(512, 512, 512, 1)][1] == 128
    assert table[(512, 512, 512, 0)][1] == 103
    assert table[(1024, 1024, 1024, 0)][1] == 171
    assert table[(1024, 1024, 128, 0)][1] == 128
    assert table[(256, 256, 256, 0)][1] == 128
    assert table[(256, 256, 256, 1)][1] == 43
    # a lattice shorter than 32 planes is one chunk
    assert table[(128, 16, 12, 0)][1] == 12 and table[(64, 8, 8, 1)][1] == 8
    # never more than 192 planes
    assert all(cz <= 192 for _, cz, _ in table.values())
    # values given by the caller are kept
    assert keep == (4, 7)


def test_chunks_for_batched_work_lists(rules):
    """Work lists of the batched launch aim at about 2048 blocks per realization:
    FP64 512^3 takes ceil(2048 / 824) = 3 chunks of 171 planes, 1024^3 the 192-plane cap
    (6 chunks of 171), 256^3 FP32 (4 x 29 = 116 tiles) the 32-plane floor (8 chunks)."""
    table, _ = rules
    assert table[(512, 512, 512, 1)][2] == 171
    assert table[(1024, 1024, 1024, 1)][2] == 171
    assert table[(256, 256, 256, 0)][2] == 32
