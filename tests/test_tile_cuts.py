"""Host-side check of the sink-tile cut the force work list uses (no GPU).

The cut is compiled from the library's own header into a small host program.  Invariants: the tiles of a cell
partition its sinks in order; a tile holds at most G*S sinks in G groups of L lanes with L*G <= 64 and
L <= max_lanes; whole 64-group tiles come first; every tile but a cell's last fills its wave (G*L = 64, G*S
sinks); the last one keeps at least 7/8 of the lanes busy unless its group count is a power of two or a further
cut would need more than max_lanes lanes per group; and a cell never takes more
than g/64 + 1 + rest/11 tiles (rest = g mod 64 groups), the bound the work-list capacity is sized by.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def cuts(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("cuts") / "tile_cuts")
    r = subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "tile_cuts_main.cpp")], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    rows = []
    for line in out.splitlines():
        f = line.split()
        n, S, ml, c = map(int, f[:4])
        tiles = [tuple(map(int, x.split(","))) for x in f[4:]]
        assert len(tiles) == c
        rows.append((n, S, ml, tiles))
    return rows


def test_tiles_partition_the_sinks(cuts):
    for n, S, ml, tiles in cuts:
        t = 0
        for L, G, t0, nt in tiles:
            assert t0 == t and 0 < nt <= G * S, (n, S, ml, tiles)
            assert 1 <= L <= ml and L * G <= 64, (n, S, ml, tiles)
            t += nt
        assert t == n, (n, S, ml, tiles)


def test_whole_tiles_first_and_every_tile_but_the_last_fills_its_wave(cuts):
    for n, S, ml, tiles in cuts:
        g = (n + S - 1) // S
        for k, (L, G, t0, nt) in enumerate(tiles):
            if k < g // 64:
                assert (L, G) == (1, 64), (n, S, ml, tiles)
            if k < len(tiles) - 1:
                assert L * G == 64 and nt == G * S, (n, S, ml, tiles)
        L, G, t0, nt = tiles[-1]
        groups = (nt + S - 1) // S
        k = 1 << (groups.bit_length() - 1)     # the largest power of two <= groups
        if k != groups and 64 // k <= ml:
            assert 8 * groups * L >= 7 * 64, (n, S, ml, tiles)


def test_tile_count_bound_of_the_work_list_capacity(cuts):
    for n, S, ml, tiles in cuts:
        g = (n + S - 1) // S
        assert len(tiles) <= g // 64 + 1 + (g % 64) / 11, (n, S, ml, tiles)


def test_example_from_the_description(cuts):
    # 43 groups of one sink: 32 with 2 lanes each, 8 with 8, 3 with 21
    row = [r for r in cuts if r[:3] == (43, 1, 64)][0]
    assert [(L, G, nt) for L, G, t0, nt in row[3]] == [(2, 32, 32), (8, 8, 8), (21, 3, 3)]
