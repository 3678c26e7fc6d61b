"""Host logic of the 3-D blocked launch that needs no GPU: how many z
segments each tile column is split into.  A small host program that includes
the kernel header is compiled with hipcc and run on the CPU; it calls only
the segment-length chooser (no device code runs).

The chooser models a launch as rounds of `resident` equal work-groups, each
loading its segment plus 2H planes, and takes the fewest segments within 3%
of the model's best, with segments no shorter than 4H planes (and 8)."""
import math
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include "wh_block3d_impl.h"
#include <cstdio>
int main() {
  int nz, H, resident;
  long long tiles;
  while (std::scanf("%d %lld %d %d", &nz, &tiles, &H, &resident) == 4)
    std::printf("%d\n", wh::block3d_zlen(nz, tiles, H, resident));
  return 0;
}
"""


def _model(nz, tiles, H, resident):
    """The same choice written out from its definition."""
    planes = nz + 1
    min_len = max(4 * H, 8)
    max_seg = max(planes // min_len, 1)

    def cost(n):
        length = -(-planes // n)
        segs = -(-planes // length)
        rounds = -(-(tiles * segs) // resident)
        return rounds * (length + 2 * H), length

    best = min(cost(n)[0] for n in range(1, max_seg + 1))
    for n in range(1, max_seg + 1):
        c, length = cost(n)
        if c <= 1.03 * best:
            return length


@pytest.fixture(scope="module")
def zlen(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("launch_shape")
    src, exe = d / "zlen.hip", d / "zlen"
    src.write_text(PROGRAM)
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2504_03074_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)

    def run(cases):
        text = "".join(f"{nz} {t} {h} {r}\n" for nz, t, h, r in cases)
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
        return [int(x) for x in out.split()]
    return run


def _tiles(n, ox=56, oy=24):
    return math.ceil((n + 1) / ox) * math.ceil((n + 1) / oy)


def test_cube_shapes(zlen):
    """512^3 (FP32, 2nd order, K = 4: 220 tile columns on 256 CUs) runs one
    segment per column; 1024^3 three; the 130 x 61 x 45 grid of the parity
    tests two; a grid thinner than one segment one."""
    cases = [(512, _tiles(512), 4, 256), (1024, _tiles(1024), 4, 256), (45, 9, 4, 256), (8, 1, 4, 256)]
    got = zlen(cases)
    segments = [math.ceil((nz + 1) / z) for (nz, _, _, _), z in zip(cases, got)]
    assert segments == [1, 3, 2, 1]


def test_matches_the_model_and_its_bounds(zlen):
    """Over a spread of grids, halos and device sizes the chooser returns the
    model's choice, and no segment is shorter than max(4H, 8) planes unless
    the whole column is."""
    cases = []
    for nz in (4, 17, 45, 64, 129, 257, 513, 1025, 2049):
        for tiles in (1, 9, 55, 220, 817, 3182):
            for H in (1, 2, 3, 4, 6):
                for resident in (256, 512):
                    cases.append((nz, tiles, H, resident))
    got = zlen(cases)
    for (nz, tiles, H, resident), z in zip(cases, got):
        assert z == _model(nz, tiles, H, resident), (nz, tiles, H, resident, z)
        planes = nz + 1
        assert 1 <= z <= planes
        if planes >= max(4 * H, 8):
            assert z >= max(4 * H, 8), (nz, tiles, H, resident, z)
