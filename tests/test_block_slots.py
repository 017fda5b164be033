"""The halo blocks of the block engines (paper_2004_13475_amd/csrc/
block_slots.inc): the committed file is what its generator writes, and every
8 x 8 block that holds a member within D steps of some 64 x 64 tile of a real
gasket is listed (found here by a different method: repeated dilation of
each tile's members over the whole array, four or eight neighbours)."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2004_13475_amd", "csrc")


def halo_lists():
    text = open(os.path.join(CSRC, "block_slots.inc")).read()
    out = {}
    for name, depth, body in re.findall(r"kHalo_(\w+?)_(\d+)\[\]\[2\] = \{(.*)\};", text):
        out[(name, int(depth))] = {(int(a), int(b)) for a, b in re.findall(r"\{(-?\d+), (-?\d+)\}", body)}
    return out


def test_generator_matches_committed_file():
    r = subprocess.run([sys.executable, os.path.join(CSRC, "gen_block_slots.py"), "--check"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def reached_blocks(k, moore, depth):
    """Blocks (relative to each tile's first block) holding a member within
    `depth` steps of the tile, over all non-empty tiles of the level-k gasket."""
    n = 1 << k
    x = np.arange(n)
    mem = (x[None, :] & x[:, None]) == 0  # [y, x]
    out = set()
    pad = depth + 1
    for ty in range(n >> 6):
        for tx in range(n >> 6):
            if tx & ty:
                continue
            # a window of the tile and `pad` cells around it (the array's
            # edge closes it: cells beyond are not members)
            y0, y1 = max(0, ty * 64 - pad), min(n, ty * 64 + 64 + pad)
            x0, x1 = max(0, tx * 64 - pad), min(n, tx * 64 + 64 + pad)
            m = mem[y0:y1, x0:x1]
            cur = np.zeros_like(m)
            cur[ty * 64 - y0:ty * 64 + 64 - y0, tx * 64 - x0:tx * 64 + 64 - x0] = \
                m[ty * 64 - y0:ty * 64 + 64 - y0, tx * 64 - x0:tx * 64 + 64 - x0]
            for _ in range(depth):
                g = cur.copy()
                g[1:, :] |= cur[:-1, :]
                g[:-1, :] |= cur[1:, :]
                g[:, 1:] |= cur[:, :-1]
                g[:, :-1] |= cur[:, 1:]
                if moore:
                    g[1:, 1:] |= cur[:-1, :-1]
                    g[:-1, :-1] |= cur[1:, 1:]
                    g[1:, :-1] |= cur[:-1, 1:]
                    g[:-1, 1:] |= cur[1:, :-1]
                cur = g & m
            ys, xs = np.nonzero(cur)
            bx = (xs + x0) // 8 - tx * 8
            by = (ys + y0) // 8 - ty * 8
            out |= set(zip(bx.tolist(), by.tolist()))
    return {b for b in out if not (0 <= b[0] < 8 and 0 <= b[1] < 8)}


@pytest.mark.parametrize("name,moore,depth", [("heat", False, 16), ("heat", False, 24),
                                              ("heat", False, 32), ("moore", True, 16),
                                              ("moore", True, 24)])
def test_halo_lists_hold_every_reachable_block(name, moore, depth):
    lists = halo_lists()
    listed = lists[(name, depth)]
    assert len(listed) <= 63 - 27, "27 tile blocks, the halo and a free zero lane fit 64 lanes"
    for b in listed:  # listed blocks are non-empty within their tile
        assert ((b[0] % 8) & (b[1] % 8)) == 0, b
    found = reached_blocks(10, moore, depth)
    assert found <= listed, sorted(found - listed)
    # nothing listed is unreachable at level 10 (the list is the union, not a box)
    assert listed == found, sorted(listed - found)
