"""GPU parity of compact storage through lambda^-1: pack / unpack and the
compact seeded fill against the oracle's layout, compact steps against the
steps over the n x n array (bit for bit) and the oracle, and a level-18
gasket (beyond the n x n array's range) sampled against oracle windows."""
import numpy as np
import pytest

import fractal_inputs as fi
import oracle
import paper_2004_13475_amd as F
from gpu_util import (ALPHA, assert_match, oracle_steps, to_device, torch_dev, window_plan,
                      zeros_state)

pytestmark = pytest.mark.gpu

RULES = [fi.RULE_CA, fi.RULE_HEAT]
STEPS = (1, 2, 3, 7, 8, 13, 16, 19, 32, 37)


def _sync():
    torch_dev().cuda.synchronize()


def _rs(rule):
    """Tile levels compact storage takes for the rule (16-byte tile rows)."""
    return range(4, 8) if rule == fi.RULE_CA else range(2, 8)


def _cbuf(k, r, rule):
    torch = torch_dev()
    nbytes = F.compact_bytes(k, r, rule)
    return torch.zeros(nbytes // (1 if rule == fi.RULE_CA else 4),
                       dtype=torch.uint8 if rule == fi.RULE_CA else torch.float32, device="cuda")


@pytest.mark.parametrize("rule", RULES)
def test_pack_unpack_and_seed_match_oracle(rule):
    for k in range(2, 12):
        st = fi.full_state(k, rule, 40 + k)
        emb = to_device(st)
        for r in _rs(rule):
            if r > k:
                continue
            c = _cbuf(k, r, rule)
            F.pack(k, r, rule, emb, c)
            want = oracle.pack(k, r, st)
            back = zeros_state(k, rule)
            F.unpack(k, r, rule, c, back)
            s = _cbuf(k, r, rule)
            F.compact_seed_fill(k, r, rule, 40 + k, s)
            _sync()
            assert np.array_equal(c.cpu().numpy().view(np.uint8), want.view(np.uint8)), (k, r)
            assert np.array_equal(back.cpu().numpy().view(np.uint8), st.view(np.uint8)), (k, r)
            assert np.array_equal(s.cpu().numpy().view(np.uint8), want.view(np.uint8)), (k, r)


def _valid(rule, r, T):
    rho = 1 << r
    if rule == fi.RULE_CA:
        return T <= 16
    # heat: 1, 2 or 4 halo lanes of 4 cells per side for up to 4, 8 or 16
    # steps; 16-step heat launches need tiles of side >= 16
    hl_cells = 4 if T <= 4 else (8 if T <= 8 else 16)
    return T <= 16 and T <= rho and hl_cells <= rho


BLOCK = F.FLAG_BLOCK | F.FLAG_SEGMENTS


@pytest.mark.parametrize("rule", RULES)
def test_compact_step_equals_array_step(rule):
    """Compact steps (every tile size, 1..16 march steps per launch, the
    block engine on 64 x 64 tiles with 16 to 36 steps per launch -- the
    default there -- both store kinds, step counts that exercise the
    power-of-two tail and the parity split) give exactly the packed result
    of the same steps over the n x n array; small levels also against the
    oracle."""
    torch = torch_dev()
    fl_list = [0, F.FLAG_NT_STORE, F.FLAG_FUSE2, F.FLAG_FUSE4 | F.FLAG_NT_STORE, F.FLAG_FUSE8,
               F.FLAG_FUSE16, BLOCK | F.FLAG_FUSE16, BLOCK | F.FLAG_FUSE24 | F.FLAG_NT_STORE,
               BLOCK | F.FLAG_FUSE36]
    for k in (4, 6, 8, 11):
        init = fi.window_values(k, rule, 80 + k)
        for r in _rs(rule):
            if r > k:
                continue
            refs = {}
            for steps in STEPS:
                a0, a1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, a0, a1, steps, r, 64, 2,
                             F.FLAG_SEGMENTS)
                c = _cbuf(k, r, rule)
                F.pack(k, r, rule, a0 if steps % 2 == 0 else a1, c)
                _sync()
                refs[steps] = c.view(torch.uint8).clone()
            for fl in fl_list:
                T = 16 if fl & F.FLAG_FUSE16 else 8 if fl & F.FLAG_FUSE8 else \
                    4 if fl & F.FLAG_FUSE4 else 2 if fl & F.FLAG_FUSE2 else 1
                ok = (r == 6) if fl & F.FLAG_BLOCK else (fl == 0 or _valid(rule, r, T))
                if not ok:
                    with pytest.raises(F.FractalError) as e:
                        F.compact_step(k, r, rule, ALPHA, _cbuf(k, r, rule), _cbuf(k, r, rule),
                                       4, fl)
                    assert e.value.code == F.E_INVAL
                    continue
                for steps in STEPS + ((72, 73) if fl & F.FLAG_BLOCK or r == 6 else ()):
                    if steps not in refs:
                        a0, a1 = to_device(init), zeros_state(k, rule)
                        F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, a0, a1, steps, r, 64, 2,
                                     F.FLAG_SEGMENTS)
                        c = _cbuf(k, r, rule)
                        F.pack(k, r, rule, a0 if steps % 2 == 0 else a1, c)
                        _sync()
                        refs[steps] = c.view(torch.uint8).clone()
                    c0, c1 = _cbuf(k, r, rule), _cbuf(k, r, rule)
                    F.pack(k, r, rule, to_device(init), c0)
                    F.compact_step(k, r, rule, ALPHA, c0, c1, steps, fl)
                    _sync()
                    got = (c0 if steps % 2 == 0 else c1).view(torch.uint8)
                    assert torch.equal(got, refs[steps]), (k, r, fl, steps)
            if k <= 8:
                c0, c1 = _cbuf(k, r, rule), _cbuf(k, r, rule)
                F.pack(k, r, rule, to_device(init), c0)
                F.compact_step(k, r, rule, ALPHA, c0, c1, 19)
                _sync()
                emb = oracle.unpack(k, r, c1.cpu().numpy())
                ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), 19)
                assert_match(k, rule, emb, ref, f"compact k={k} r={r}")


@pytest.mark.parametrize("rule,k", [(fi.RULE_CA, 18), (fi.RULE_HEAT, 18), (fi.RULE_CA, 20)])
def test_compact_level18_sampled(rule, k):
    """Level 18 (387,420,489 cells; the n x n array would take 69 GB per
    float32 buffer) and, for the automaton, level 20 (3.5e9 cells, 19.6 GB
    per compact state, byte offsets past 2^34): 64 compact steps from the
    compact seeded fill (the block engine on 64 x 64 tiles; heat at level 18
    also on 32 x 32 tiles with the march), sampled in light-cone windows
    against the oracle."""
    torch = torch_dev()
    for r in ((6,) if rule == fi.RULE_CA else (6, 5)):
        _sampled(rule, k, r)


def _sampled(rule, k, r):
    torch = torch_dev()
    steps = 64
    n = 1 << k
    c0, c1 = _cbuf(k, r, rule), _cbuf(k, r, rule)
    F.compact_seed_fill(k, r, rule, 7, c0)
    F.compact_step(k, r, rule, ALPHA, c0, c1, steps)
    _sync()
    flat = c0  # steps even: result in buffer 0
    for (cx, cy) in [(0, 0), (n - 48, 0), (0, n - 48), (150000, 40000), (65536, 131072),
                     (n // 2 + 4096, n // 4 + 12)]:
        x0, y0, w, h = window_plan(k, steps, 48, 48, cx, cy)
        win = fi.window_values(k, rule, 7, x0, y0, w, h)
        ref = oracle_steps(k, rule, win if rule == 0 else win.astype(np.float64), steps, x0, y0)
        rs, cs = oracle.valid_interior(k, x0, y0, w, h, steps)
        ref = ref[rs, cs]
        ys, xs = np.meshgrid(np.arange(y0 + rs.start, y0 + rs.start + ref.shape[0]),
                             np.arange(x0 + cs.start, x0 + cs.start + ref.shape[1]),
                             indexing="ij")
        live = ((xs >> r) & (ys >> r)) == 0
        got = np.zeros(ref.shape, dtype=ref.dtype if rule == 0 else np.float32)
        idx = torch.from_numpy(oracle.compact_index(k, r, xs[live], ys[live])).to("cuda")
        got[live] = flat[idx].cpu().numpy()
        assert_match(k, rule, got, ref, f"compact k{k} window ({cx},{cy})")
    del c0, c1
    torch.cuda.empty_cache()


def test_compact_rejects_bad_arguments():
    torch = torch_dev()
    a, b = _cbuf(8, 4, fi.RULE_CA), _cbuf(8, 4, fi.RULE_CA)
    bad = [
        lambda: F.compact_step(8, 3, fi.RULE_CA, ALPHA, a, b, 2),          # 8-byte rows
        lambda: F.compact_step(21, 4, fi.RULE_CA, ALPHA, a, b, 2),         # level > 20
        lambda: F.compact_step(8, 4, fi.RULE_CA, ALPHA, a, a, 2),          # aliasing
        lambda: F.compact_step(8, 4, fi.RULE_CA, ALPHA, a, b, 2, 1 << 9),  # unknown flag
        lambda: F.compact_step(8, 1, fi.RULE_HEAT, ALPHA, a, b, 2),        # 8-byte rows
        lambda: F.compact_step(8, 2, fi.RULE_HEAT, ALPHA, a, b, 2, F.FLAG_FUSE8),  # T > rho
        lambda: F.pack(17, 4, fi.RULE_CA, a, b),                           # array level > 16
        lambda: F.compact_step(8, 4, fi.RULE_CA, ALPHA, a, b, 2, BLOCK | F.FLAG_FUSE16),  # r != 6
        lambda: F.compact_step(8, 6, fi.RULE_CA, ALPHA, a, b, 2,
                               BLOCK | F.FLAG_MARCH | F.FLAG_FUSE16),       # two engines
    ]
    for f in bad:
        with pytest.raises(F.FractalError) as e:
            f()
        assert e.value.code == F.E_INVAL
    del torch
