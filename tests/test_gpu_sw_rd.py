"""GPU parity of tests SW (single write) and RD (reduction) of Section 6.2
on the lambda and bounding-box maps, against the CPU oracle, through the C
ABI."""
import numpy as np
import pytest

import fractal_inputs as fi
import oracle
import paper_2004_13475_amd as F
from gpu_util import ALPHA, to_device, torch_dev, zeros_state

pytestmark = pytest.mark.gpu

RULES = [fi.RULE_CA, fi.RULE_HEAT]
MAPS = [F.MAP_LAMBDA, F.MAP_BB]
VALUES = {fi.RULE_CA: 0x5A, fi.RULE_HEAT: 0x40490FDB}  # 90, float32(pi)


def _sync():
    torch_dev().cuda.synchronize()


def _rd(map_, k, r, rule, buf):
    torch = torch_dev()
    work = torch.empty(max(8, F.reduce_workspace(k, r)), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int64 if rule == fi.RULE_CA else torch.float64,
                      device="cuda")
    F.reduce(map_, k, r, rule, buf, work, out)
    _sync()
    return int(out.item()) if rule == fi.RULE_CA else float(out.item())


@pytest.mark.parametrize("map_", MAPS)
@pytest.mark.parametrize("rule", RULES)
def test_single_write_every_tile_size(rule, map_):
    """SW on a zeroed buffer gives the oracle's array bit for bit, for every
    level up to 11 and every tile size."""
    torch = torch_dev()
    for k in range(0, 12):
        want = oracle.single_write(k, rule, VALUES[rule])
        for r in range(0, min(k, 7) + 1):
            if k - r > 15:
                continue
            buf = zeros_state(k, rule)
            F.single_write(map_, k, r, rule, VALUES[rule], buf)
            _sync()
            got = buf.cpu().numpy()
            assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (k, r, map_)
    del torch


@pytest.mark.parametrize("rule", RULES)
def test_single_write_leaves_memberless_segments(rule):
    """Off-gasket cells are 0 where they lie in a non-empty tile and a 64-byte
    segment that holds a member, and keep their old bytes elsewhere."""
    torch = torch_dev()
    k, r = 9, 4
    n = 1 << k
    s = 1 if rule == fi.RULE_CA else 4
    seg = 64 // s
    buf = torch.full((n, n), 7, dtype=torch.uint8 if rule == fi.RULE_CA else torch.float32,
                     device="cuda")
    F.single_write(F.MAP_LAMBDA, k, r, rule, VALUES[rule], buf)
    _sync()
    got = buf.cpu().numpy()
    mask = oracle.gasket_mask(k)
    want_on = oracle.single_write(k, rule, VALUES[rule])
    assert np.array_equal(got[mask], want_on[mask])
    ys, xs = np.nonzero(~mask)
    live = (((xs // seg) & (ys // seg)) == 0) & (((xs >> r) & (ys >> r)) == 0)
    off = got[ys, xs]
    assert np.all(off[live] == 0)
    assert np.all(off[~live] == 7)
    del torch


@pytest.mark.parametrize("map_", MAPS)
@pytest.mark.parametrize("rule", RULES)
def test_reduce_seeded_states_exact(rule, map_):
    """RD of seeded states equals the oracle exactly (uint8: integers;
    float32: multiples of 2^-24, whose float64 sum is exact), for levels up
    to 12 and every tile size; lambda and BB agree bit for bit."""
    for k in range(0, 13):
        st = fi.full_state(k, rule, 30 + k)
        want = oracle.reduce_(k, st)
        buf = to_device(st)
        for r in range(0, min(k, 7) + 1):
            if k - r > 15:
                continue
            got = _rd(map_, k, r, rule, buf)
            assert got == want, (k, r, map_, got, want)


def test_reduce_evolved_heat_within_bound_and_map_independent():
    """After 37 heat steps the values are no longer on a 2^-24 grid: RD is
    within 1e-12 (relative) of the exactly rounded sum, identical between
    lambda and BB, tile sizes and repeated calls, and off-gasket garbage does
    not count."""
    torch = torch_dev()
    k = 11
    init = fi.window_values(k, fi.RULE_HEAT, 5)
    b0, b1 = to_device(init), zeros_state(k, fi.RULE_HEAT)
    F.lambda_step(k, F.R_AUTO, fi.RULE_HEAT, ALPHA, b0, b1, 37)
    _sync()
    state = b1.cpu().numpy()
    want = oracle.reduce_(k, state)
    seen = set()
    for map_ in MAPS:
        for r in (2, 4, 5, 7):
            for _ in range(2):
                got = _rd(map_, k, r, fi.RULE_HEAT, b1)
                assert abs(got - want) <= 1e-12 * abs(want), (map_, r, got, want)
                seen.add((r, got))
    # one value per tile size: the map and the repetition do not change bits
    assert len({g for (_, g) in seen}) <= 4
    by_r = {}
    for (r, g) in seen:
        by_r.setdefault(r, set()).add(g)
    assert all(len(v) == 1 for v in by_r.values())
    # garbage off the gasket is ignored
    mask = torch.from_numpy(~oracle.gasket_mask(k)).to("cuda")
    b1[mask] = 1234.5
    assert _rd(F.MAP_LAMBDA, k, 5, fi.RULE_HEAT, b1) == by_r[5].pop()
    del torch


@pytest.mark.parametrize("rule", RULES)
def test_sw_then_rd_full_size_k16(rule):
    """Level 16 (43,046,721 members): SW of a value then RD gives exactly
    3^16 times the value, through both maps."""
    torch = torch_dev()
    k, r = 16, 5
    buf = zeros_state(k, rule)
    F.single_write(F.MAP_LAMBDA, k, r, rule, VALUES[rule], buf)
    _sync()
    cell = 0x5A if rule == fi.RULE_CA else float(np.array([VALUES[rule]], np.uint32).view(np.float32)[0])
    for map_ in MAPS:
        got = _rd(map_, k, r, rule, buf)
        want = (3 ** k) * cell
        if rule == fi.RULE_CA:
            assert got == want
        else:
            # 3^16 values of one float32: each partial sum is a small integer
            # multiple of it, exact in float64
            assert got == float(np.float64(cell) * (3 ** k))
    del buf
    torch.cuda.empty_cache()


def test_sw_rd_reject_bad_arguments():
    torch = torch_dev()
    buf = zeros_state(6, fi.RULE_CA)
    for args in [(2, 6, 3), (0, 17, 3), (0, 6, 8), (0, 6, 7)]:
        with pytest.raises(F.FractalError):
            F.single_write(args[0], args[1], args[2], fi.RULE_CA, 1, buf)
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(F.FractalError):
        F.reduce(F.MAP_LAMBDA, 6, 2, fi.RULE_CA, buf, small, out)
    del torch
