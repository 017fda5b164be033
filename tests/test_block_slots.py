"""The halo blocks of the block engines (paper_2004_13475_amd/csrc/
block_slots.inc): the committed file is what its generator writes; the masks
of non-empty neighbouring tiles it lists are all that occur in gasket tile
arrays of 1 to 4096 tiles a side; and, tile by tile over a real gasket, the
list of the tile's mask holds every 8 x 8 block with a member within D steps
of the tile and nothing else (found here by a different method than the
generator's breadth-first search over masks: repeated dilation of each
tile's members over the whole array, four or eight neighbours)."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2004_13475_amd", "csrc")
VARIANTS = ([(f"heat_{d}", False, d, 64) for d in (16, 24, 32, 36)] +
            [(f"moore_{d}", True, d, 64) for d in (16, 24, 32, 36)] +
            [("heat_36_t128", False, 36, 128), ("moore_36_t128", True, 36, 128)])


def parse():
    text = open(os.path.join(CSRC, "block_slots.inc")).read()
    index = [int(v) for v in re.search(r"kMaskIndex\[64\] = \{([^}]*)\}", text).group(1).split(",")]
    lists = {}
    for name, body in re.findall(r"kHalo_(\w+)\[\d+\]\[\d+\]\[2\] = \{(.*?)\};", text, re.S):
        counts = [int(v) for v in re.search(rf"kHaloCount_{name}\[\d+\] = \{{([^}}]*)\}}",
                                            text).group(1).split(",")]
        rows = re.findall(r"\{((?:\{-?\d+, -?\d+\}(?:, )?)+)\}", body)
        assert len(rows) == len(counts)
        per = []
        for row, c in zip(rows, counts):
            pts = [(int(a), int(b)) for a, b in re.findall(r"\{(-?\d+), (-?\d+)\}", row)]
            per.append(set(pts[:c]))
            assert len(set(pts[:c])) == c
        lists[name] = per
    return index, lists


def tile_masks(nt):
    """Mask of non-empty neighbouring tiles (bit 0 left, 1 above, 2 right, 3
    below, 4 above right, 5 below left) of every tile of an nt x nt array;
    -1 for empty tiles."""
    t = np.arange(nt, dtype=np.int64)
    tx, ty = t[None, :], t[:, None]

    def present(dx, dy):
        x, y = tx + dx, ty + dy
        return (x >= 0) & (x < nt) & (y >= 0) & (y < nt) & ((x & y) == 0)

    m = np.zeros((nt, nt), dtype=np.int64)
    for bit, (dx, dy) in enumerate(((-1, 0), (0, -1), (1, 0), (0, 1), (1, -1), (-1, 1))):
        m |= present(dx, dy).astype(np.int64) << bit
    return np.where((tx & ty) == 0, m, -1)


def test_generator_matches_committed_file():
    r = subprocess.run([sys.executable, os.path.join(CSRC, "gen_block_slots.py"), "--check"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_every_occurring_mask_is_listed():
    index, _ = parse()
    listed = {m for m in range(64) if index[m] >= 0}
    every = set()
    for j in range(13):
        seen = set(np.unique(tile_masks(1 << j)).tolist()) - {-1}
        assert seen <= listed, (1 << j, sorted(seen - listed))
        every |= seen
    assert every == listed
    assert index[0] >= 0  # the lone tile of a level-6 array


def reached_blocks(k, moore, depth, tile=64):
    """Per non-empty tile (tx, ty) (side `tile`) of the level-k gasket: the
    blocks outside it (relative to its first block) holding a member within
    `depth` steps."""
    n = 1 << k
    x = np.arange(n)
    mem = (x[None, :] & x[:, None]) == 0  # [y, x]
    out = {}
    pad = depth + 1
    T = tile
    for ty in range(n // T):
        for tx in range(n // T):
            if tx & ty:
                continue
            y0, y1 = max(0, ty * T - pad), min(n, ty * T + T + pad)
            x0, x1 = max(0, tx * T - pad), min(n, tx * T + T + pad)
            m = mem[y0:y1, x0:x1]
            cur = np.zeros_like(m)
            sy, sx = slice(ty * T - y0, ty * T + T - y0), slice(tx * T - x0, tx * T + T - x0)
            cur[sy, sx] = m[sy, sx]
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
            bx = (xs + x0) // 8 - tx * (T // 8)
            by = (ys + y0) // 8 - ty * (T // 8)
            out[(tx, ty)] = {b for b in zip(bx.tolist(), by.tolist())
                             if not (0 <= b[0] < T // 8 and 0 <= b[1] < T // 8)}
    return out


@pytest.mark.parametrize("name,moore,depth,tile", VARIANTS)
def test_halo_lists_are_exactly_the_reachable_blocks(name, moore, depth, tile):
    index, lists = parse()
    per_mask = lists[name]
    k = 10 if tile == 64 else 11
    masks = tile_masks((1 << k) // tile)
    union = [set() for _ in per_mask]
    for (tx, ty), found in reached_blocks(k, moore, depth, tile).items():
        i = index[int(masks[ty, tx])]
        assert i >= 0
        assert found <= per_mask[i], ((tx, ty), sorted(found - per_mask[i]))
        union[i] |= found
    inside = 27 if tile == 64 else 81  # non-empty blocks of the tile
    slots = 64 if tile == 64 else 128  # one or two blocks per lane
    for i, listed in enumerate(per_mask):
        assert len(listed) <= slots - 1 - inside, "the tile, the halo and a free zero slot fit"
        for b in listed:  # listed blocks are non-empty within their tile
            assert ((b[0] % 8) & (b[1] % 8)) == 0, b
        assert union[i] == listed, (i, sorted(listed - union[i]))
