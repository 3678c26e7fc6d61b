"""Host logic of the 3-D launches that needs no GPU: how many z segments each
tile column of the blocked kernel is split into, and the XCD-contiguous
numbering of the first step's work-groups.  Small host programs that include
the kernel headers are compiled with hipcc and run on the CPU; they call only
host functions (no device code runs).

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


XCD_PROGRAM = r"""
#include "wh_xcd.h"
#include <cstdio>
#include <vector>
int main() {
  long long nblk;
  while (std::scanf("%lld", &nblk) == 1) {
    const dim3 g = wh::xcd_grid(nblk);
    const long long total = (long long)g.x * g.y;
    std::vector<unsigned char> seen((size_t)nblk, 0);
    long long dup = 0, missing = 0;
    for (long long L = 0; L < total; ++L) {
      const long long lb = wh::xcd_block(L, total);
      if (lb < nblk && seen[(size_t)lb]++) ++dup;
    }
    for (long long b = 0; b < nblk; ++b) missing += !seen[(size_t)b];
    std::printf("%u %u %lld %lld\n", g.x, g.y, dup, missing);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def xcd(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("xcd_grid")
    src, exe = d / "xcd.hip", d / "xcd"
    src.write_text(XCD_PROGRAM)
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", os.path.join(ROOT, "paper_2504_03074_amd", "csrc"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)

    def run(nblks):
        text = "".join(f"{n}\n" for n in nblks)
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
        return [tuple(int(x) for x in line.split()) for line in out.splitlines()]
    return run


def test_xcd_numbering_covers_every_block_once(xcd):
    """Every logical block gets exactly one work-group, for one-row grids and
    for the rows of 2^16 work-groups past 2^24 blocks (the 512^3 first step:
    9 x 129 x 129 blocks); every row is a multiple of 8 work-groups and at
    most 2^26 of them (64 work-items each, 2^32 per launch dimension)."""
    nblks = [1, 7, 8, 9, 1000, 9 * 129 * 129, (1 << 24) - 3, (1 << 24) + 5, 3 * (1 << 24) + 1]
    for n, (gx, gy, dup, missing) in zip(nblks, xcd(nblks)):
        assert dup == 0 and missing == 0, n
        assert gx % 8 == 0 and gx * 64 <= 1 << 32, n
        assert gx * gy >= n and gx * gy - n < max(8, gx), n
        assert (gy == 1) == (n <= 1 << 24), n
