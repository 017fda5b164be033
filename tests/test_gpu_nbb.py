"""GPU parity of the general NBB family (Section 3, Table 1): Theorem 1's
map for every built-in table, and tests SW, RD and CA over every tile size
through lambda and the bounding box, against the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_2004_13475_amd as F
from gpu_util import torch_dev

pytestmark = pytest.mark.gpu

BUILTINS = [F.NBB_GASKET, F.NBB_CARPET, F.NBB_VICSEK, F.NBB_XFRACTAL, F.NBB_HFRACTAL,
            F.NBB_CANTOR]
MAPS = [F.MAP_LAMBDA, F.MAP_BB]


def _sync():
    torch_dev().cuda.synchronize()


def _dev(arr):
    return torch_dev().from_numpy(np.ascontiguousarray(arr)).to("cuda")


@pytest.mark.parametrize("which", BUILTINS)
def test_nbb_lambda_map_matches_oracle(which):
    torch = torch_dev()
    f = F.nbb_builtin(which)
    reps = f.replicas()
    for rb in range(0, 8 if f.k <= 5 else 6):
        gx, gy = f.k ** ((rb + 1) // 2), f.k ** (rb // 2)
        out = torch.zeros(2 * gx * gy, dtype=torch.int32, device="cuda")
        F.nbb_lambda_map(f, rb, out)
        _sync()
        got = out.cpu().numpy().reshape(gy, gx, 2)
        for wy in range(gy):
            for wx in range(gx):
                assert tuple(got[wy, wx]) == oracle.nbb_lambda(reps, f.s, rb, wx, wy), \
                    (which, rb, wx, wy)


def _levels(f):
    return (8,) if f.s == 2 else (4, 5)


@pytest.mark.parametrize("map_", MAPS)
@pytest.mark.parametrize("which", BUILTINS)
def test_nbb_sw_rd_ca_every_tile_size(which, map_):
    """SW on a zeroed array, RD of a random state with garbage off the
    fractal, and 5 automaton steps checked one by one, for every tile side
    s^r <= 128."""
    torch = torch_dev()
    f = F.nbb_builtin(which)
    reps = f.replicas()
    rng = np.random.default_rng(100 + which)
    for level in _levels(f):
        n = f.s ** level
        mask = oracle.nbb_member_mask(reps, f.s, level)
        want_sw = oracle.nbb_single_write(reps, f.s, level, 0xA7)
        junk = rng.integers(0, 256, size=(n, n), dtype=np.uint8)
        want_rd = oracle.nbb_reduce(reps, f.s, level, junk)
        life = (rng.random((n, n)) < 0.5).astype(np.uint8) * mask
        for r in range(0, level + 1):
            if f.s ** r > 128:
                break
            buf = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
            F.nbb_single_write(f, map_, level, r, 0xA7, buf)
            _sync()
            assert np.array_equal(buf.cpu().numpy(), want_sw), (which, level, r, "SW")
            work = torch.empty(max(8, F.nbb_reduce_workspace(f, level, r)), dtype=torch.uint8,
                               device="cuda")
            out = torch.zeros(1, dtype=torch.int64, device="cuda")
            F.nbb_reduce(f, map_, level, r, _dev(junk), work, out)
            _sync()
            assert int(out.item()) == want_rd, (which, level, r, "RD")
            b0, b1 = _dev(life), torch.zeros((n, n), dtype=torch.uint8, device="cuda")
            ref = life
            for t in range(1, 6):
                src, dst = (b0, b1) if t % 2 == 1 else (b1, b0)
                F.nbb_ca_step(f, map_, level, r, src, dst, 1)
                _sync()
                ref = oracle.nbb_ca_run(reps, f.s, level, ref, 1)
                assert np.array_equal(dst.cpu().numpy(), ref), (which, level, r, "CA", t)


def test_nbb_carpet_level9_sampled():
    """Sierpinski carpet at level 9 (19683 x 19683, 134,217,728 members):
    12 automaton steps through lambda with 27 x 27 tiles, sampled in
    light-cone windows against the oracle; the bounding box gives the same
    array."""
    torch = torch_dev()
    f = F.nbb_builtin(F.NBB_CARPET)
    reps = f.replicas()
    level, r, steps = 9, 3, 12
    n = 3 ** level
    rng = np.random.default_rng(9)
    st = (rng.random((n, n), dtype=np.float32) < 0.5).astype(np.uint8)
    st &= oracle.nbb_member_mask(reps, 3, level).astype(np.uint8)
    b0, b1 = _dev(st), torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    F.nbb_ca_step(f, F.MAP_LAMBDA, level, r, b0, b1, steps)
    c0, c1 = _dev(st), torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    F.nbb_ca_step(f, F.MAP_BB, level, r, c0, c1, steps)
    _sync()
    assert torch.equal(b0, c0)
    for (cx, cy) in [(0, 0), (n - 40, n - 40), (9000, 3000), (6561, 13122)]:
        x0, y0 = max(0, cx - steps), max(0, cy - steps)
        x1, y1 = min(n, cx + 40 + steps), min(n, cy + 40 + steps)
        ref = oracle.nbb_ca_run(reps, 3, level, st[y0:y1, x0:x1], steps, x0, y0)
        rs, cs = oracle.valid_interior(30, x0, y0, x1 - x0, y1 - y0, steps)
        # valid_interior treats edges at 0 and 2^30; clip to this array's edge
        hi_y = (y1 - y0) if y1 >= n else (y1 - y0) - steps
        hi_x = (x1 - x0) if x1 >= n else (x1 - x0) - steps
        rs, cs = slice(rs.start, hi_y), slice(cs.start, hi_x)
        got = b0[y0:y1, x0:x1].cpu().numpy()[rs, cs]
        assert np.array_equal(got, ref[rs, cs]), (cx, cy)
    del b0, b1, c0, c1
    torch.cuda.empty_cache()


def test_nbb_rejects_bad_tables():
    torch = torch_dev()
    buf = torch.zeros((9, 9), dtype=torch.uint8, device="cuda")
    bad = [F.nbb_make(2, 3, [(0, 0), (0, 0)]),      # overlapping replicas
           F.nbb_make(2, 3, [(0, 0), (3, 0)]),      # offset outside the grid
           F.nbb_make(5, 2, [(0, 0)] * 5),          # more replicas than cells
           F.nbb_make(2, 9, [(0, 0), (1, 0)])]      # scale beyond 8
    for f in bad:
        with pytest.raises(F.FractalError) as e:
            F.nbb_single_write(f, F.MAP_LAMBDA, 2, 0, 1, buf)
        assert e.value.code == F.E_INVAL
    f = F.nbb_builtin(F.NBB_CARPET)
    with pytest.raises(F.FractalError):
        F.nbb_single_write(f, F.MAP_LAMBDA, 2, 5, 1, buf)   # r > level
    with pytest.raises(F.FractalError):
        F.nbb_single_write(f, F.MAP_LAMBDA, 11, 2, 1, buf)  # n > 65536
    with pytest.raises(F.FractalError):
        F.nbb_single_write(f, F.MAP_LAMBDA, 6, 5, 1, buf)   # tile 243 > 128
    del torch
