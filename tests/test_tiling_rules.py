"""Tiling rules of the banded inner solver, on the CPU.

The host and the kernels share the rules in csrc/sg_internal.h: how many
64-lane regions tile a grid row (each region holds its tile's interior plus a
halo of h nodes on every side that is not the grid's edge), how many tiles
the busiest block of the automatic grid works per phase, and which band height
a launch with few tiles takes. A small program prints the library's values
(tests/host_tiling/tiling_rules.cpp, built with g++); they are checked here
against the geometry a region must satisfy, placed tile by tile, and against
the rows the busiest block sweeps for each candidate height."""

import itertools
import math
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"


@pytest.fixture(scope="module")
def rules(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(f"{ROCM}/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path_factory.mktemp("tiling") / "tiling_rules")
    src = os.path.join(HERE, "host_tiling", "tiling_rules.cpp")
    res = subprocess.run([gxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
                          f"-I{os.path.join(ROOT, 'include')}", "-o", exe, src], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]

    def run(cases):
        text = "".join(" ".join(map(str, c)) + "\n" for c in cases)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [tuple(int(x) for x in line.split()) for line in out.splitlines()]
    return run


def halo(degree):
    # the Chebyshev halo (degree - 1 nodes, at least one) plus one node
    return max(degree - 1, 1) + 1


def place_tiles(nx, h):
    """Tiles of a grid row, placed left to right: the first region starts at
    the grid's left edge and the last ends at its right edge, so those tiles
    need the halo on one side only; every other region needs it on both."""
    if nx <= 64:
        return [(0, nx)]
    tiles, x = [], 0
    while nx - x > 64 - h:                     # the rest does not fit an edge tile
        w = 64 - h if x == 0 else 64 - 2 * h
        tiles.append((x, x + w))
        x += w
    tiles.append((x, nx))
    return tiles


def region_holds(nx, h, tiles):
    if nx <= 64:                               # one region from the left edge over the whole row
        return tiles == [(0, nx)]
    for i, (a, b) in enumerate(tiles):
        r0 = 0 if i == 0 else (nx - 64 if i == len(tiles) - 1 else a - h)
        lo = a if i == 0 else a - h            # halo needed left of the tile
        hi = b if i == len(tiles) - 1 else b + h
        if not (0 <= r0 <= lo and hi <= r0 + 64 <= nx):
            return False
    return True


def busiest(nwork, ncu):
    """Tiles of the busiest block: one tile per block if they fit the compute
    units, else two per block on at most ncu blocks, the work list cut into
    even contiguous shares."""
    grid = nwork if nwork <= ncu else min((nwork + 1) // 2, ncu)
    sizes = [(b + 1) * nwork // grid - b * nwork // grid for b in range(grid)]
    assert sum(sizes) == nwork
    return max(sizes)


def band_rows(nx, degree, prec, ncols, ncu):
    default = 256 if prec == 32 else 128
    heights = [256, 128, 64] if prec == 32 else [128, 64]
    tiles = lambda rows: ncols * len(place_tiles(nx, halo(degree))) * math.ceil(nx / rows)  # noqa: E731
    if tiles(default) >= ncu:
        return default
    cost = {r: busiest(tiles(r), ncu) * (r + 2 * halo(degree)) for r in heights}
    best = min(cost.values())
    return min(r for r in heights if cost[r] == best)   # the shorter on a tie


CASES = list(itertools.product([3, 32, 63, 64, 65, 96, 97, 128, 129, 200, 255, 299, 511],
                               [1, 2, 3, 8, 12, 16], [32, 64], [1, 3, 10, 55, 220], [256, 80]))


def test_tiling_rules_match_the_geometry(rules):
    got = rules(CASES)
    assert len(got) == len(CASES)
    for (nx, d, prec, ncols, ncu), (h, ntx, ntx_a, rows, busy) in zip(CASES, got):
        case = (nx, d, prec, ncols, ncu)
        assert h == halo(d), case
        tiles = place_tiles(nx, h)
        assert region_holds(nx, h, tiles), case
        assert ntx == len(tiles), case
        assert ntx_a == len(place_tiles(nx, 1)), case
        assert rows == band_rows(nx, d, prec, ncols, ncu), case
        assert busy == busiest(ncols * ntx * math.ceil(nx / rows), ncu), case


def test_benchmark_launches(rules):
    """The launches of one preconditioner action on 255 x 255 unknowns at
    degree 16 and 256 compute units (columns per level: 1, 10, 55, 220)."""
    got = rules([(255, 16, prec, ncols, 256) for prec in (64, 32) for ncols in (1, 10, 55, 220)])
    rows = [g[3] for g in got]
    busy = [g[4] for g in got]
    assert [g[1] for g in got] == [7] * 8 and [g[2] for g in got] == [5] * 8
    assert rows == [64, 128, 128, 128, 64, 128, 256, 256]
    # level 2 in FP64: 770 tiles take four on the busiest block; level 3's
    # 3080 tiles would take 13 on the automatic grid (whole columns: 14)
    assert busy == [1, 1, 4, 13, 1, 1, 2, 7]
