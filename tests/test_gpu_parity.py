"""GPU parity: lambda map, seeded fill, lambda / bounding-box / matrix-core
steps against the CPU oracle, through the C ABI (ctypes binding)."""
import numpy as np
import pytest

import fractal_inputs as fi
import oracle
import paper_2004_13475_amd as F
from gpu_util import (ALPHA, assert_match, heat_err, oracle_steps, to_device,
                      torch_dev, window_plan, zeros_state)

pytestmark = pytest.mark.gpu

RULES = [fi.RULE_CA, fi.RULE_HEAT]
MAPS = [F.MAP_LAMBDA, F.MAP_BB, F.MAP_MFMA]


def _sync():
    torch_dev().cuda.synchronize()


# ------------------------------------------------------------------ map
@pytest.mark.parametrize("mfma", [False, True])
def test_lambda_map_all_levels(mfma):
    torch = torch_dev()
    for rb in range(0, 13):
        for r in (0, 3):
            k = rb + r
            gx, gy = F.grid_dims(k, r)
            out = torch.zeros(gx * gy * 2, dtype=torch.int32, device="cuda")
            (F.lambda_map_mfma if mfma else F.lambda_map)(k, r, out)
            _sync()
            got = out.cpu().numpy().view(np.uint32).reshape(gy, gx, 2)
            want = oracle.lambda_grid(rb)
            assert np.array_equal(got, want), f"rb={rb} r={r} mfma={mfma}"


@pytest.mark.parametrize("mfma", [False, True])
def test_lambda_map_large_levels_sampled(mfma):
    torch = torch_dev()
    rng = np.random.default_rng(5)
    levels = [13, 14, 15, 16] if mfma else [13, 14, 15, 16, 17, 18]
    for rb in levels:
        gx, gy = F.grid_dims(rb, 0)
        out = torch.zeros(gx * gy * 2, dtype=torch.int32, device="cuda")
        (F.lambda_map_mfma if mfma else F.lambda_map)(rb, 0, out)
        _sync()
        got = out.cpu().numpy().view(np.uint32).reshape(gy, gx, 2)
        for _ in range(3000):
            wx, wy = int(rng.integers(gx)), int(rng.integers(gy))
            assert tuple(got[wy, wx]) == oracle.lambda_(rb, wx, wy)
        # bijection onto X & Y == 0 over the whole grid
        flat = got.reshape(-1, 2).astype(np.int64)
        assert np.all((flat[:, 0] & flat[:, 1]) == 0)
        keys = flat[:, 1] * (1 << rb) + flat[:, 0]
        assert np.unique(keys).size == gx * gy


def test_lambda_map_rejects_bad_levels():
    torch = torch_dev()
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(F.FractalError):
        F.lambda_map_mfma(17, 0, out)
    with pytest.raises(F.FractalError):
        F.lambda_map(3, 4, out)


# ------------------------------------------------------------------ seed
@pytest.mark.parametrize("rule", RULES)
def test_seed_fill_matches_input_generator(rule):
    for k in (0, 1, 2, 3, 4, 5, 9, 11):
        buf = zeros_state(k, rule)
        buf.fill_(7 if rule == fi.RULE_CA else 3.0)
        F.seed_fill(k, rule, 1234 + k, buf)
        _sync()
        want = fi.window_values(k, rule, 1234 + k)
        got = buf.cpu().numpy()
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), f"k={k}"


# ------------------------------------------------------------------ steps
def _run(map_, k, r, rule, b0, b1, steps, flags=None):
    alpha = ALPHA
    if flags is not None:
        t = F.get_tuning(k, rule) if r == F.R_AUTO else (r, 64, 2, 0)
        F.step_tuned(map_, k, rule, alpha, b0, b1, steps, t[0], t[1], t[2], flags)
    elif map_ == F.MAP_LAMBDA:
        F.lambda_step(k, r, rule, alpha, b0, b1, steps)
    elif map_ == F.MAP_BB:
        F.bb_step(k, r, rule, alpha, b0, b1, steps)
    else:
        F.lambda_step_mfma(k, r, rule, alpha, b0, b1, steps)


@pytest.mark.parametrize("flags", [None, 1, 2, 3])
@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("map_", MAPS)
def test_steps_small_levels_every_r(rule, map_, flags):
    """Every tile size and launch flag on small gaskets, checked after each
    of 6 steps."""
    for k in range(0, 9):
        for r in range(0, min(k, 7) + 1):
            init = fi.window_values(k, rule, 100 + k)
            b0 = to_device(init)
            b1 = zeros_state(k, rule)
            ref = init if rule == fi.RULE_CA else init.astype(np.float64)
            for t in range(1, 7):
                # one step from the current buffer into the other
                src, dst = (b0, b1) if (t - 1) % 2 == 0 else (b1, b0)
                _run(map_, k, r, rule, src, dst, 1, flags)
                _sync()
                ref = oracle_steps(k, rule, ref, 1)
                assert_match(k, rule, dst.cpu().numpy(), ref,
                             f"map={map_} k={k} r={r} t={t}")


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_steps_k10_checkpoints(rule, r):
    """Level 10 (n = 1024, 59049 cells): every step up to 32, then 100, for
    lambda and bounding box, against the whole-array oracle."""
    k = 10
    init = fi.window_values(k, rule, 77)
    bufs = {m: (to_device(init), zeros_state(k, rule)) for m in (F.MAP_LAMBDA, F.MAP_BB)}
    ref = init if rule == fi.RULE_CA else init.astype(np.float64)
    t = 0
    for target in list(range(1, 33)) + [100]:
        dt = target - t
        ref = oracle_steps(k, rule, ref, dt)
        for m, (b0, b1) in bufs.items():
            _run(m, k, r, rule, b0, b1, dt)
            _sync()
            res = b0 if dt % 2 == 0 else b1
            assert_match(k, rule, res.cpu().numpy(), ref, f"map={m} r={r} t={target}")
            if dt % 2 == 1:
                bufs[m] = (b1, b0)
        t = target


@pytest.mark.parametrize("rule", RULES)
def test_lambda_bb_mfma_bit_identical_k12(rule):
    torch = torch_dev()
    k, steps = 12, 9
    init = fi.window_values(k, rule, 5)
    outs = []
    for m in MAPS:
        for (r, th, order, fl) in [(3, 64, 0, 0), (4, 64, 2, 1), (5, 256, 1, 2), (6, 256, 2, 3),
                                   (5, 64, 0, 1), (2, 64, 2, 3), (1, 64, 0, 1), (7, 256, 0, 3),
                                   (7, 64, 2, 1), (5, 256, 0, 11), (6, 64, 2, 19),
                                   (7, 256, 1, 17)]:
            b0, b1 = to_device(init), zeros_state(k, rule)
            F.step_tuned(m, k, rule, ALPHA, b0, b1, steps, r, th, order, fl)
            _sync()
            outs.append(((m, r, th, order, fl), b1.cpu().numpy()))
    base = outs[0][1]
    for cfg, o in outs[1:]:
        assert np.array_equal(o.view(np.uint8), base.view(np.uint8)), f"{cfg} differs"
    ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), steps)
    assert_match(k, rule, base, ref, "k12")
    del torch


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("map_", MAPS)
def test_fused_launches(rule, map_):
    """Two or four steps per launch (halo rows and an extra chunk column
    staged, intermediate steps in LDS) give the same bits as one step per
    launch, for every fusable tile size and step counts that exercise the
    paired launches and the single-step tail; small levels also against the
    oracle."""
    torch = torch_dev()
    cell = 1 if rule == fi.RULE_CA else 4
    for k in (5, 8, 11):
        init = fi.window_values(k, rule, 60 + k)
        for r in range(0, min(k, 7) + 1):
            if (1 << r) * cell < 16 or k - r > 15:
                continue
            th = 256 if r >= 4 else 64
            for steps in (1, 4, 5, 8, 11, 16, 19):
                for fl in (9, 11, 17, 19):
                    a0, a1 = to_device(init), zeros_state(k, rule)
                    F.step_tuned(map_, k, rule, ALPHA, a0, a1, steps, r, th, 2, fl)
                    b0, b1 = to_device(init), zeros_state(k, rule)
                    F.step_tuned(map_, k, rule, ALPHA, b0, b1, steps, r, th, 2, fl & ~24)
                    _sync()
                    fa = a0 if steps % 2 == 0 else a1
                    fb = b0 if steps % 2 == 0 else b1
                    assert torch.equal(fa.view(torch.uint8), fb.view(torch.uint8)), \
                        (k, r, steps, fl)
                    if k <= 8 and fl in (11, 19):
                        ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64),
                                           steps)
                        assert_match(k, rule, fa.cpu().numpy(), ref, f"fused k={k} r={r} t={steps}")


MARCH_FUSE = (0, F.FLAG_FUSE2, F.FLAG_FUSE4, F.FLAG_FUSE8, F.FLAG_FUSE16)


@pytest.mark.parametrize("map_", [F.MAP_LAMBDA, F.MAP_BB])
@pytest.mark.parametrize("rule", RULES)
def test_march_launches(rule, map_):
    """The register-march engine (1, 2, 4 or 8 steps per launch, tiles side
    by side in a wavefront, bands of rows) gives the same bits as one step
    per launch of the LDS engine, for every tile size it takes, every order,
    both workgroup sizes and step counts that exercise the power-of-two tail
    and the parity split; small levels also against the oracle."""
    torch = torch_dev()
    cell = 1 if rule == fi.RULE_CA else 4
    for k in (4, 6, 8, 11):
        init = fi.window_values(k, rule, 70 + k)
        for r in range(0, min(k, 7) + 1):
            if (1 << r) * cell < 16 or k - r > 15:
                continue
            ref_by_steps = {}
            for steps in (1, 2, 3, 7, 8, 13, 16, 19, 32, 37):
                b0, b1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(map_, k, rule, ALPHA, b0, b1, steps, r, 64, 2, F.FLAG_SEGMENTS)
                _sync()
                ref_by_steps[steps] = (b0 if steps % 2 == 0 else b1).view(torch.uint8).clone()
            for fuse in MARCH_FUSE:
                if fuse == F.FLAG_FUSE16 and rule != fi.RULE_CA and r < 4:
                    continue  # heat marches 16 steps on tiles of side >= 16 only
                for (th, order, nt) in ((256, 2, 2), (64, 0, 0), (256, 1, 0)):
                    fl = F.FLAG_MARCH | F.FLAG_SEGMENTS | nt | fuse
                    for steps in (1, 2, 3, 7, 8, 13, 16, 19, 32, 37):
                        a0, a1 = to_device(init), zeros_state(k, rule)
                        F.step_tuned(map_, k, rule, ALPHA, a0, a1, steps, r, th, order, fl)
                        _sync()
                        fa = a0 if steps % 2 == 0 else a1
                        assert torch.equal(fa.view(torch.uint8), ref_by_steps[steps]), \
                            (k, r, steps, fl, th, order)
            if k <= 8:
                fl = F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_NT_STORE | F.FLAG_FUSE8
                a0, a1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(map_, k, rule, ALPHA, a0, a1, 19, r, 256, 2, fl)
                _sync()
                ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), 19)
                assert_match(k, rule, a1.cpu().numpy(), ref, f"march k={k} r={r}")


@pytest.mark.parametrize("rule", RULES)
def test_march_launch_plan_every_step_count(rule):
    """Sixteen-step lambda tunings split a call into launches of 16, 12, 10,
    8, 4, 2 and 1 steps by a cost model (20 -> 10 + 10, 30 -> 10 + 10 + 8 +
    2), with a launch count of the parity of the step count.  Every step
    count 1..40 at every tile size (the 10- and 12-step kernels exist for
    sides 16..64; side 128 keeps powers of two), single tiles and stacks of
    two, both store kinds, gives the same bits as one step per launch; level
    9 also against the oracle."""
    torch = torch_dev()
    k = 9
    init = fi.window_values(k, rule, 77)
    cur, nxt = to_device(init), zeros_state(k, rule)
    refs = {0: cur.view(torch.uint8).clone()}
    for t in range(1, 41):
        F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, cur, nxt, 1, 4, 64, 2, F.FLAG_SEGMENTS)
        cur, nxt = nxt, cur
        _sync()
        refs[t] = cur.view(torch.uint8).clone()
    for r in range(4, 8):
        for extra in (0, F.FLAG_NT_STORE, F.FLAG_STACK2):
            fl = F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_FUSE16 | extra
            for steps in range(1, 41):
                a0, a1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, a0, a1, steps, r, 256, 2, fl)
                _sync()
                fa = a0 if steps % 2 == 0 else a1
                assert torch.equal(fa.view(torch.uint8), refs[steps]), (r, extra, steps)
    ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), 27)
    a0, a1 = to_device(init), zeros_state(k, rule)
    F.lambda_step(k, F.R_AUTO, rule, ALPHA, a0, a1, 27)
    _sync()
    assert_match(k, rule, a1.cpu().numpy(), ref, "even split, 27 steps")


@pytest.mark.parametrize("map_", [F.MAP_LAMBDA, F.MAP_BB])
@pytest.mark.parametrize("rule", RULES)
def test_block_engine_every_step_count(rule, map_):
    """The block engine (64 x 64 tiles: one wavefront per tile, one lane per
    non-empty 8 x 8 block of the tile and of the part of its halo that can
    reach it; heat cells in registers, automaton cells as a 64-bit board)
    gives the same bits as one step per launch of the LDS engine for every
    step count 1..40 (1..72 for the 24-, 32- and 36-step launches), every
    launch cap (FUSE2 .. FUSE36, or none: one step per launch), every
    dispatch order and both store kinds, at levels 6 (one tile, the halo
    outside the array), 7, 9 and 12, on 64 x 64 tiles and (from level 7)
    128 x 128 tiles with two blocks per lane; level 9 also against the
    oracle."""
    torch = torch_dev()
    BLOCK = F.FLAG_BLOCK | F.FLAG_SEGMENTS
    deep = [F.FLAG_FUSE24, F.FLAG_FUSE32, F.FLAG_FUSE36]
    for k in (6, 7, 9, 12):
        init = fi.window_values(k, rule, 60 + k)
        cur, nxt = to_device(init), zeros_state(k, rule)
        refs = {}
        for t in range(1, 73):
            F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, cur, nxt, 1, min(k, 4), 64, 2,
                         F.FLAG_SEGMENTS)
            cur, nxt = nxt, cur
            _sync()
            refs[t] = cur.view(torch.uint8).clone()
        cases = [(F.FLAG_FUSE16, 2, 0, 6), (F.FLAG_FUSE16, 0, F.FLAG_NT_STORE, 6),
                 (F.FLAG_FUSE16, 1, 0, 6), (F.FLAG_FUSE8, 2, F.FLAG_NT_STORE, 6),
                 (F.FLAG_FUSE4, 2, 0, 6), (F.FLAG_FUSE2, 0, 0, 6), (0, 2, 0, 6)]
        cases += [(d, 2, 0, 6) for d in deep] + [(d, 1, F.FLAG_NT_STORE, 6) for d in deep]
        if k >= 7:
            # the two-slot form on 128 x 128 tiles
            cases += [(F.FLAG_FUSE36, 1, 0, 7), (F.FLAG_FUSE16, 0, F.FLAG_NT_STORE, 7),
                      (F.FLAG_FUSE24, 2, 0, 7)]
        for fuse, order, nt, r in cases:
            if fuse in deep and r == 6:
                step_list = range(1, 73) if (order == 2 and nt == 0) else (1, 23, 24, 25, 33, 36, 47, 65)
            elif r == 7:
                step_list = range(1, 73) if fuse == F.FLAG_FUSE36 else (1, 15, 16, 17, 24, 25, 49)
            elif fuse == F.FLAG_FUSE16 and order == 2:
                step_list = range(1, 41)
            else:
                step_list = (1, 2, 3, 7, 16, 17, 33)
            for steps in step_list:
                a0, a1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(map_, k, rule, ALPHA, a0, a1, steps, r, 256, order,
                             BLOCK | fuse | nt)
                _sync()
                fa = a0 if steps % 2 == 0 else a1
                assert torch.equal(fa.view(torch.uint8), refs[steps]), (k, fuse, order, nt, r, steps)
        if k == 9:
            ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), 27)
            a0, a1 = to_device(init), zeros_state(k, rule)
            F.step_tuned(map_, k, rule, ALPHA, a0, a1, 27, 6, 256, 2, BLOCK | F.FLAG_FUSE16)
            _sync()
            assert_match(k, rule, a1.cpu().numpy(), ref, "block engine, 27 steps")
            ref = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), 61)
            for d, r in [(d, 6) for d in deep] + [(F.FLAG_FUSE36, 7)]:
                a0, a1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(map_, k, rule, ALPHA, a0, a1, 61, r, 256, 2, BLOCK | d)
                _sync()
                assert_match(k, rule, a1.cpu().numpy(), ref, f"block engine flags {d} r {r}, 61 steps")


@pytest.mark.parametrize("rule", RULES)
def test_block_engine_full_size_k16_equals_march(rule):
    """Level 16, the whole array: the block engine (lambda map; 16-, 24- and
    36-step launches) gives the same bits as the register march on 64 x 64
    tiles after 1, 16, 37 and 64 steps, and its bounding-box form the same
    as its lambda form."""
    torch = torch_dev()
    k = 16
    n = 1 << k
    dt = torch.uint8 if rule == fi.RULE_CA else torch.float32
    deep = F.FLAG_FUSE36
    for steps in (1, 16, 37, 64):
        outs = []
        runs = [(F.MAP_LAMBDA, F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE16 | F.FLAG_NT_STORE, 6),
                (F.MAP_LAMBDA, F.FLAG_BLOCK | F.FLAG_SEGMENTS | deep, 6),
                (F.MAP_LAMBDA, F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE24 | F.FLAG_NT_STORE, 6),
                (F.MAP_BB, F.FLAG_BLOCK | F.FLAG_SEGMENTS | deep, 6),
                (F.MAP_LAMBDA, F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_FUSE16, 6)]
        runs += [(F.MAP_LAMBDA, F.FLAG_BLOCK | F.FLAG_SEGMENTS | deep, 7),  # 128 x 128 tiles
                 (F.MAP_BB, F.FLAG_BLOCK | F.FLAG_SEGMENTS | deep, 7)]
        for map_, fl, r in runs:
            b0 = torch.empty((n, n), dtype=dt, device="cuda")
            b1 = torch.zeros_like(b0)
            F.seed_fill(k, rule, 5, b0)
            F.step_tuned(map_, k, rule, ALPHA, b0, b1, steps, r, 256, 2, fl)
            _sync()
            res = b1 if steps % 2 else b0
            if outs:
                assert torch.equal(res.view(torch.uint8), outs[0].view(torch.uint8)), (steps, fl, r)
            else:
                outs.append(res)
            del b0, b1
        del outs
        torch.cuda.empty_cache()


@pytest.mark.parametrize("rule", RULES)
def test_march_stacks(rule):
    """Stacks of up to 2, 4 or 8 tiles (each class of equal column runs a
    smaller gasket of stacks under lambda) give the same bits as one step
    per launch, at levels where the stack level is clamped to the tile
    level (k - r < 3) and above; small levels also against the oracle."""
    torch = torch_dev()
    cell = 1 if rule == fi.RULE_CA else 4
    fuses = (F.FLAG_FUSE2, F.FLAG_FUSE8, F.FLAG_FUSE16)
    for k in (4, 6, 9, 12):
        init = fi.window_values(k, rule, 90 + k)
        for r in range(2, min(k, 7) + 1):
            if (1 << r) * cell < 16:
                continue
            for steps in (3, 16, 37):
                b0, b1 = to_device(init), zeros_state(k, rule)
                F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, b0, b1, steps, r, 64, 2,
                             F.FLAG_SEGMENTS)
                _sync()
                ref = (b0 if steps % 2 == 0 else b1).view(torch.uint8).clone()
                for stack in (F.FLAG_STACK2, F.FLAG_STACK4, F.FLAG_STACK8):
                    for fuse in fuses:
                        if fuse == F.FLAG_FUSE16 and rule != fi.RULE_CA and r < 4:
                            continue
                        fl = F.FLAG_MARCH | F.FLAG_SEGMENTS | fuse | stack
                        a0, a1 = to_device(init), zeros_state(k, rule)
                        F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, a0, a1, steps, r, 256, 2, fl)
                        _sync()
                        fa = a0 if steps % 2 == 0 else a1
                        assert torch.equal(fa.view(torch.uint8), ref), (k, r, steps, fl)
                if k <= 6 and steps == 37:
                    want = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64),
                                        steps)
                    assert_match(k, rule, (b0 if steps % 2 == 0 else b1).cpu().numpy(), want,
                                 f"stacks k={k} r={r}")


@pytest.mark.parametrize("rule", RULES)
def test_autotune_picks_a_valid_launch(rule):
    """The autotuner times its candidates (the LDS, march and block engines,
    fusion depths, stacks) on the caller's buffers, caches the fastest for the level, and
    lambda steps under that cached launch give the same bits as one step per
    launch; the built-in default comes back after set_tuning restores it."""
    torch = torch_dev()
    k = 10
    before = F.get_tuning(k, rule)
    init = fi.window_values(k, rule, 123)
    w0, w1 = to_device(init), zeros_state(k, rule)
    t = F.autotune(k, rule, ALPHA, w0, w1)
    _sync()
    assert tuple(F.get_tuning(k, rule)) == tuple(t)
    r, th, order, fl = t
    assert 0 <= r <= 7 and th in (64, 256) and order in (0, 1, 2)
    assert fl & ~(1 | 2 | 8 | 16 | 32 | 64 | 128 | 256 | 512 | 1024 | 2048 | 4096 | 8192 |
                  16384 | 32768) == 0
    for steps in (5, 40):
        a0, a1 = to_device(init), zeros_state(k, rule)
        F.lambda_step(k, F.R_AUTO, rule, ALPHA, a0, a1, steps)
        b0, b1 = to_device(init), zeros_state(k, rule)
        F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, b0, b1, steps, r, 64, 2, F.FLAG_SEGMENTS)
        _sync()
        got = a0 if steps % 2 == 0 else a1
        ref = b0 if steps % 2 == 0 else b1
        assert torch.equal(got.view(torch.uint8), ref.view(torch.uint8)), (t, steps)
    F.set_tuning(k, rule, *before)
    assert tuple(F.get_tuning(k, rule)) == tuple(before)


@pytest.mark.parametrize("rule", RULES)
def test_march_other_occupancy_bit_identical(rule):
    """The long march launches compiled for the other occupancy
    (FRACTAL_FLAG_OCC_ALT, a dimension of the autotuner) give the bits of
    the default kernels, on every tile size that has them (and are ignored
    where none exists), with non-temporal stores and stacks."""
    torch = torch_dev()
    k = 12
    init = fi.window_values(k, rule, 55)
    fuses = (F.FLAG_FUSE8, F.FLAG_FUSE16)
    for r in range(2 if rule == fi.RULE_HEAT else 4, 8):
        for fuse in fuses:
            if fuse == F.FLAG_FUSE16 and rule != fi.RULE_CA and r < 4:
                continue
            for extra in (0, F.FLAG_NT_STORE, F.FLAG_STACK2):
                fl = F.FLAG_MARCH | F.FLAG_SEGMENTS | fuse | extra
                for steps in (16, 21):
                    a0, a1 = to_device(init), zeros_state(k, rule)
                    F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, a0, a1, steps, r, 256, 2, fl)
                    b0, b1 = to_device(init), zeros_state(k, rule)
                    F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, b0, b1, steps, r, 256, 2,
                                 fl | F.FLAG_OCC_ALT)
                    _sync()
                    fa = a0 if steps % 2 == 0 else a1
                    fb = b0 if steps % 2 == 0 else b1
                    assert torch.equal(fa.view(torch.uint8), fb.view(torch.uint8)), \
                        (r, fl, steps)


def test_march_rejects_bad_tunings():
    """March launches need whole segments, rows of >= 16 bytes and a lambda
    or BB map; FUSE8 needs the march engine."""
    torch = torch_dev()
    b0, b1 = zeros_state(6, fi.RULE_CA), zeros_state(6, fi.RULE_CA)
    bad = [
        (F.MAP_LAMBDA, 4, F.FLAG_MARCH),                                   # no SEGMENTS
        (F.MAP_LAMBDA, 3, F.FLAG_MARCH | F.FLAG_SEGMENTS),                 # 8-byte rows
        (F.MAP_MFMA, 4, F.FLAG_MARCH | F.FLAG_SEGMENTS),                   # no march form
        (F.MAP_LAMBDA, 4, F.FLAG_SEGMENTS | F.FLAG_FUSE8),                 # FUSE8 without march
        (F.MAP_LAMBDA, 4, F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_FUSE2 | F.FLAG_FUSE8),
    ]
    for map_, r, fl in bad:
        with pytest.raises(F.FractalError) as e:
            F.step_tuned(map_, 6, fi.RULE_CA, ALPHA, b0, b1, 4, r, 64, 0, fl)
        assert e.value.code == F.E_INVAL, (map_, r, fl)
    del torch


@pytest.mark.parametrize("flags", [11, 19, 35 | 16, 35 | 64, 35 | 128, 35 | 128 | 256,
                                   35 | 64 | 512])
@pytest.mark.parametrize("rule", RULES)
def test_fused_full_size_k16_sampled(rule, flags):
    """Level 16 with two-, four-, eight- and sixteen-step launches (LDS and
    register march engines, single tiles and stacks of 2 or 4; heat's
    sixteen-step launches on 64 x 64 tiles), 200 steps, sampled against the
    oracle's light-cone windows."""
    k = 16
    n = 1 << k
    r = 7 if rule == fi.RULE_CA else 6
    torch = torch_dev()
    b0, b1 = zeros_state(k, rule), zeros_state(k, rule)
    F.seed_fill(k, rule, 3, b0)
    boxes = [(0, 0, 32, 32), (n - 32, 0, 32, 32), (30000, 20000, 32, 32)]
    plans = []
    for (cx, cy, w, h) in boxes:
        x0, y0, ww, hh = window_plan(k, 200, w, h, cx, cy)
        win = fi.window_values(k, rule, 3, x0, y0, ww, hh)
        plans.append(((x0, y0, ww, hh), win if rule == 0 else win.astype(np.float64)))
    F.step_tuned(F.MAP_LAMBDA, k, rule, ALPHA, b0, b1, 200, r, 256, 0, flags)
    _sync()
    for (x0, y0, ww, hh), state in plans:
        ref = oracle_steps(k, rule, state, 200, x0, y0)
        rs, cs = oracle.valid_interior(k, x0, y0, ww, hh, 200)
        ref = ref[rs, cs]
        gy0, gx0 = y0 + rs.start, x0 + cs.start
        got = b0[gy0:gy0 + ref.shape[0], gx0:gx0 + ref.shape[1]].cpu().numpy()
        assert_match(k, rule, got, ref, f"fused k16 box=({x0},{y0})")
    del torch


@pytest.mark.parametrize("rule", RULES)
def test_off_gasket_stays_zero_and_steps0_noop(rule):
    torch = torch_dev()
    k = 11
    init = fi.window_values(k, rule, 8)
    b0, b1 = to_device(init), zeros_state(k, rule)
    F.lambda_step(k, 4, rule, ALPHA, b0, b1, 0)
    _sync()
    assert torch.equal(b0.cpu(), torch.from_numpy(init))
    F.lambda_step(k, 4, rule, ALPHA, b0, b1, 5)
    _sync()
    mem = torch.from_numpy(fi.member_mask(k)).cuda()
    assert not bool((b1.to(torch.float32)[~mem] != 0).any())


# ---------------------------------------------------------- full sizes
def _full_size_check(k, rule, r, checkpoints, boxes, map_=F.MAP_LAMBDA, seed=1):
    """Seed on the GPU, run to each checkpoint, and compare sampled boxes
    with the oracle run on light-cone windows of the CPU-generated input."""
    torch = torch_dev()
    b0, b1 = zeros_state(k, rule), zeros_state(k, rule)
    F.seed_fill(k, rule, seed, b0)
    tmax = checkpoints[-1]
    plans = []
    for (cx, cy, w, h) in boxes:
        x0, y0, ww, hh = window_plan(k, tmax, w, h, cx, cy)
        win = fi.window_values(k, rule, seed, x0, y0, ww, hh)
        state = win if rule == fi.RULE_CA else win.astype(np.float64)
        plans.append([(cx, cy, w, h), (x0, y0, ww, hh), state])
    t = 0
    cur, other = b0, b1
    for target in checkpoints:
        dt = target - t
        _run(map_, k, r, rule, cur, other, dt)
        if dt % 2 == 1:
            cur, other = other, cur
        _sync()
        for plan in plans:
            (cx, cy, w, h), (x0, y0, ww, hh), state = plan
            state = oracle_steps(k, rule, state, dt, x0, y0)
            plan[2] = state
            rs, cs = oracle.valid_interior(k, x0, y0, ww, hh, target)
            ref = state[rs, cs]
            gy0, gx0 = y0 + rs.start, x0 + cs.start
            got = cur[gy0:gy0 + ref.shape[0], gx0:gx0 + ref.shape[1]].cpu().numpy()
            assert_match(k, rule, got, ref, f"k={k} t={target} box=({cx},{cy})")
        t = target
    del torch


@pytest.mark.parametrize("rule", RULES)
def test_full_size_k14(rule):
    """Level 14 (n = 16384, 4,782,969 cells) at the benchmark's launch
    configuration: 1000 steps, sampled at the four corners (light cones
    clipped by the array edge) and two interior boxes at early steps."""
    k = 14
    n = 1 << k
    r = F.R_AUTO  # the default launch the benchmark starts from
    _full_size_check(k, rule, r, list(range(1, 9)) + [32, 100, 1000],
                     [(0, 0, 48, 48), (n - 48, 0, 48, 48), (0, n - 48, 48, 48)])
    _full_size_check(k, rule, r, [1, 2, 3, 10, 40],
                     [(5000, 3000, 64, 64), (8192 - 20, 8192 - 20, 40, 40)])


@pytest.mark.parametrize("rule", RULES)
def test_full_size_k16(rule):
    """Level 16 (n = 65536, 43,046,721 cells, 17 GB float32 per buffer):
    200 steps, sampled boxes at corners and inside."""
    k = 16
    n = 1 << k
    r = F.R_AUTO
    _full_size_check(k, rule, r, [1, 2, 50, 200],
                     [(0, 0, 32, 32), (n - 32, 0, 32, 32), (0, n - 32, 32, 32),
                      (40000, 20000, 32, 32), (32768 - 16, 32768 - 16, 32, 32)])


@pytest.mark.parametrize("rule", RULES)
def test_max_block_level_k16(rule):
    """The largest block-space level a step accepts: k = 16 with 2 x 2 tiles
    (k - r = 15, 3^15 = 14,348,907 workgroups), two steps, sampled."""
    k, r = 16, 1
    n = 1 << k
    _full_size_check(k, rule, r, [1, 2],
                     [(0, 0, 24, 24), (n - 24, n - 24, 24, 24), (12345, 54321, 24, 24)])


def test_heat_error_metric_sane():
    a = np.array([1.0, 2.0, 0.0], dtype=np.float32)
    assert heat_err(a, a.astype(np.float64)) == 0.0


# ------------------------------------------------ per-lane map, all orders
@pytest.mark.parametrize("order", [F.ORDER_NATURAL, F.ORDER_CURVE, F.ORDER_CURVE_XCD])
def test_lambda_lane_map_matches_oracle(order):
    """The map as the register-march kernels evaluate it (one tile per lane,
    a digit loop per id) against the oracle for every block level up to 15:
    the natural order equals Theorem 1's lambda on omega = (i mod gx,
    i div gx); the curve orders are the bijection whose inverse is the
    oracle's compact index (base-3 digit mu-1 of the id is beta_mu)."""
    torch = torch_dev()
    for rb in range(0, 16):
        for r in ((0, 2) if rb <= 12 else (1,)):
            k = rb + r
            total = 3 ** rb
            out = torch.zeros(2 * total, dtype=torch.int32, device="cuda")
            F.lambda_map_tiles(k, r, order, out)
            _sync()
            got = out.cpu().numpy().view(np.uint32).reshape(total, 2).astype(np.int64)
            if order == F.ORDER_NATURAL:
                want = oracle.lambda_grid(rb).reshape(total, 2).astype(np.int64)
                assert np.array_equal(got, want), f"rb={rb}"
            else:
                assert np.all((got[:, 0] & got[:, 1]) == 0), f"rb={rb}: empty block"
                ids = oracle.compact_index(rb, 0, got[:, 0], got[:, 1])
                assert np.array_equal(ids, np.arange(total)), f"rb={rb}: not the curve order"


def test_lambda_lane_map_rejects_bad_arguments():
    torch = torch_dev()
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    for (k, r, order) in ((22, 1, 0), (3, 4, 0), (5, 1, 3)):
        with pytest.raises(F.FractalError) as e:
            F.lambda_map_tiles(k, r, order, out)
        assert e.value.code == F.E_INVAL


# ------------------------------------------- matrix-core map, auto tiles
@pytest.mark.parametrize("rule", RULES)
def test_lambda_step_mfma_auto_tile_bit_identical(rule):
    """The matrix-core lambda step at FRACTAL_R_AUTO takes the tuned tile
    size with its own (LDS-engine) launch and gives the bits of the default
    lambda step."""
    torch = torch_dev()
    for k in (10, 12):
        init = fi.window_values(k, rule, 31 + k)
        for steps in (1, 9, 20):
            a0, a1 = to_device(init), zeros_state(k, rule)
            F.lambda_step_mfma(k, F.R_AUTO, rule, ALPHA, a0, a1, steps)
            b0, b1 = to_device(init), zeros_state(k, rule)
            F.lambda_step(k, F.R_AUTO, rule, ALPHA, b0, b1, steps)
            _sync()
            fa = a0 if steps % 2 == 0 else a1
            fb = b0 if steps % 2 == 0 else b1
            assert torch.equal(fa.view(torch.uint8), fb.view(torch.uint8)), (k, steps)


# ------------------------------------------- whole arrays at full size
def _off_gasket_zero(k, buf):
    """Every cell off the gasket holds 0 (bit pattern), checked on the
    device row band by row band."""
    torch = torch_dev()
    n = 1 << k
    xs = torch.arange(n, device="cuda", dtype=torch.int64)
    step = max(1, (1 << 24) // n)
    for y0 in range(0, n, step):
        ys = torch.arange(y0, min(n, y0 + step), device="cuda", dtype=torch.int64)
        off = (ys[:, None] & xs[None, :]) != 0
        band = buf[y0:y0 + ys.numel()].view(torch.uint8 if buf.dtype == torch.uint8
                                           else torch.int32)
        if bool((band[off] != 0).any()):
            return False
    return True


@pytest.mark.parametrize("rule", RULES)
def test_full_size_k14_whole_array(rule):
    """Level 14 (n = 16384, 4,782,969 cells) at the default launch the
    benchmark uses, against the oracle over the WHOLE array: the automaton
    after every step t = 1..32 (the transient and the entry into its period-6
    attractor) and at t = 100; heat at t = 1, 10, 100, 200; every off-gasket
    cell 0 at each checkpoint."""
    k = 14
    torch = torch_dev()
    init = fi.full_state(k, rule, 9)
    cur, other = to_device(init), zeros_state(k, rule)
    ref = init if rule == fi.RULE_CA else init.astype(np.float64)
    del init
    checkpoints = list(range(1, 33)) + [100] if rule == fi.RULE_CA else [1, 10, 100, 200]
    t = 0
    for target in checkpoints:
        dt = target - t
        F.lambda_step(k, F.R_AUTO, rule, ALPHA, cur, other, dt)
        if dt % 2 == 1:
            cur, other = other, cur
        ref = oracle_steps(k, rule, ref, dt)
        _sync()
        assert_match(k, rule, cur.cpu().numpy(), ref, f"k14 whole array t={target}")
        assert _off_gasket_zero(k, cur), f"k14 t={target}: off-gasket cell not 0"
        t = target
    del torch


def _bb_lds(k, rule, b0, b1, steps):
    """The structurally different reference launch: bounding-box map, LDS
    engine, one step per launch, 32 x 32 tiles."""
    F.step_tuned(F.MAP_BB, k, rule, ALPHA, b0, b1, steps, 5, 256, F.ORDER_NATURAL,
                 F.FLAG_SEGMENTS)


@pytest.mark.parametrize("rule", RULES)
def test_full_size_k16_whole_array_lambda_equals_bb(rule):
    """Level 16 (n = 65536, 43,046,721 cells; 17 GB per float32 buffer):
    the default lambda launch (register march, lambda per lane, die-aware
    curve order, non-temporal stores) and the bounding-box LDS launch one
    step at a time give the same bits over the whole array at t = 1, 2, 16
    and 200; the off-gasket cells stay 0."""
    k = 16
    torch = torch_dev()
    lam = [zeros_state(k, rule), zeros_state(k, rule)]
    bb = [zeros_state(k, rule), zeros_state(k, rule)]
    F.seed_fill(k, rule, 21, lam[0])
    F.seed_fill(k, rule, 21, bb[0])
    t = 0
    for target in (1, 2, 16, 200):
        dt = target - t
        F.lambda_step(k, F.R_AUTO, rule, ALPHA, lam[0], lam[1], dt)
        _bb_lds(k, rule, bb[0], bb[1], dt)
        if dt % 2 == 1:
            lam.reverse()
            bb.reverse()
        _sync()
        assert torch.equal(lam[0].view(torch.uint8), bb[0].view(torch.uint8)), f"t={target}"
        t = target
    assert _off_gasket_zero(k, lam[0])
    del lam, bb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("rule", RULES)
def test_full_size_k16_full_width_bands(rule):
    """Level 16, default launch, 200 steps, against the oracle on full-width
    bands of 48 rows: across the middle of the array (row 32768 splits the
    gasket's top-level replicas, where every tile stack class and every
    die's share of the curve order meet) and across row 49152."""
    k = 16
    n = 1 << k
    steps = 200
    torch = torch_dev()
    b0, b1 = zeros_state(k, rule), zeros_state(k, rule)
    F.seed_fill(k, rule, 4, b0)
    F.lambda_step(k, F.R_AUTO, rule, ALPHA, b0, b1, steps)
    _sync()
    for cy in (32768 - 24, 49152 - 24):
        y0, h = cy - steps, 48 + 2 * steps
        win = fi.window_values(k, rule, 4, 0, y0, n, h)
        ref = oracle_steps(k, rule, win if rule == fi.RULE_CA else win.astype(np.float64),
                           steps, 0, y0)
        rs, cs = oracle.valid_interior(k, 0, y0, n, h, steps)
        assert (rs.stop - rs.start, cs.stop - cs.start) == (48, n)
        got = b0[y0 + rs.start:y0 + rs.stop].cpu().numpy()
        assert_match(k, rule, got, ref[rs, cs], f"k16 band rows {cy}..{cy + 47}")
    del b0, b1
    torch.cuda.empty_cache()


def test_heat_alpha_readings_and_underflow_k12():
    """Heat at level 12 over the whole array, one step per call for 300
    steps.  Against the oracle with alpha = (double)0.2f (the coefficient
    the GPU computes with) and with alpha = 0.2 exactly (the paper's
    value, which no float32 holds) the error metric stays <= 1e-5 at
    t = 1, 10, 100, 200.  The field decays by about 0.66 per step: the step
    at which the float32 maximum first falls below 2^-126 (subnormal) is the
    one at which the oracle's float64 maximum does (within one step: the
    threshold is crossed between roundings), and the field is exactly 0 once
    the oracle's maximum is below half the smallest subnormal (within three
    steps).  Subnormals are kept (no flush to zero)."""
    torch = torch_dev()
    k = 12
    init = fi.full_state(k, fi.RULE_HEAT, 17)
    cur, other = to_device(init), zeros_state(k, fi.RULE_HEAT)
    ref_f = init.astype(np.float64)
    ref_x = ref_f.copy()
    t_sub_gpu = t_zero_gpu = t_sub_ref = t_zero_ref = None
    errs = {}
    for t in range(1, 301):
        F.lambda_step(k, F.R_AUTO, fi.RULE_HEAT, ALPHA, cur, other, 1)
        cur, other = other, cur
        ref_f = oracle.heat_run(k, ref_f, ALPHA, 1)
        if t <= 200:
            ref_x = oracle.heat_run(k, ref_x, 0.2, 1)
        gmax = float(cur.max().item())
        rmax = float(ref_f.max())
        if t_sub_gpu is None and gmax < 2.0 ** -126:
            t_sub_gpu = t
        if t_zero_gpu is None and gmax == 0.0:
            t_zero_gpu = t
        if t_sub_ref is None and rmax < 2.0 ** -126:
            t_sub_ref = t
        if t_zero_ref is None and rmax < 2.0 ** -150:
            t_zero_ref = t
        if t in (1, 10, 100, 200):
            got = cur.cpu().numpy()
            errs[t] = (heat_err(got, ref_f), heat_err(got, ref_x))
            assert errs[t][0] <= 1e-5 and errs[t][1] <= 1e-5, (t, errs[t])
    print(f"heat k12: error vs alpha=(double)0.2f / alpha=0.2 by step {errs}; "
          f"t_underflow (float32 max < 2^-126) GPU {t_sub_gpu} oracle {t_sub_ref}; "
          f"field exactly 0 from GPU {t_zero_gpu} oracle {t_zero_ref}")
    assert t_sub_gpu is not None and abs(t_sub_gpu - t_sub_ref) <= 1
    assert t_zero_gpu is not None and abs(t_zero_gpu - t_zero_ref) <= 3
    del torch
