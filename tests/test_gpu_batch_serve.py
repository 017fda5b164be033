"""GPU tests of the batched persistent step (one HIP graph) and of the
request server: every instance / request gives the same result alone and in
the mix, and small ones match the CPU oracle."""
import time

import numpy as np
import pytest

import fractal_inputs as fi
import paper_2004_13475_amd as F
from gpu_util import ALPHA, assert_match, oracle_steps, to_device, torch_dev, zeros_state

pytestmark = pytest.mark.gpu


def _sync():
    torch_dev().cuda.synchronize()


def _alone(k, rule, steps, init):
    """The same instance through the plain lambda step entry point."""
    a0, a1 = to_device(init), zeros_state(k, rule)
    F.lambda_step(k, F.R_AUTO, rule, ALPHA, a0, a1, steps)
    return a0 if steps % 2 == 0 else a1


def _mix(count, seed, kmin, kmax, max_steps):
    rng = np.random.default_rng(seed)
    specs = []
    for j, (k, rule) in enumerate(fi.batch_instances(count, seed, kmin, kmax)):
        steps = int(rng.integers(0, max_steps + 1))
        specs.append((k, rule, steps, 1000 + j))
    return specs


MARCH = F.FLAG_MARCH | F.FLAG_SEGMENTS


@pytest.mark.parametrize("tuning", [None, (4, 64, 2, 0), (5, 64, 2, F.FLAG_PERSISTENT),
                                    (2, 64, 0, F.FLAG_PERSISTENT), (5, 256, 0, 11), (6, 0, 0, 19),
                                    (5, 64, 0, 19 | F.FLAG_PERSISTENT),
                                    (F.R_AUTO, 0, 0, MARCH | F.FLAG_FUSE8),
                                    (5, 0, 0, MARCH | F.FLAG_NT_STORE | F.FLAG_FUSE4),
                                    (4, 256, 0, MARCH | F.FLAG_FUSE2),
                                    (7, 64, 0, MARCH),
                                    (6, 0, 0, MARCH | F.FLAG_FUSE8 | F.FLAG_PERSISTENT),
                                    (5, 0, 2, MARCH | F.FLAG_FUSE16),
                                    (F.R_AUTO, 0, 0, F.FLAG_PERSISTENT),
                                    (F.R_AUTO, 0, 0, MARCH | F.FLAG_FUSE16 | F.FLAG_PERSISTENT),
                                    (6, 0, 0, F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE16),
                                    (6, 0, 1, F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE8 |
                                     F.FLAG_NT_STORE),
                                    (6, 0, 0, F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE32),
                                    (6, 0, 2, F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE36 |
                                     F.FLAG_NT_STORE)])
def test_batch_alone_equals_in_mix(tuning):
    """Every instance of a mixed batch (levels 1..11, both rules, 0..37
    steps) gives the bits of its own plain lambda step call, for per-level
    defaults, explicit tile sizes and flags, the LDS, march and block
    engines (the block engine takes heat instances of level >= 6, the others
    fall back to the march) and the persistent march grid; small ones also
    match the oracle.  The workspace is a torch-owned device buffer."""
    torch = torch_dev()
    specs = _mix(40, 3, 1, 11, 37)
    inst, inits = [], []
    for (k, rule, steps, sid) in specs:
        init = fi.window_values(k, rule, sid)
        inits.append(init)
        inst.append((k, rule, steps, ALPHA, to_device(init), zeros_state(k, rule)))
    work = torch.empty(F.batch_workspace(len(inst)), dtype=torch.uint8, device="cuda")
    F.batch_step(inst, tuning=tuning, work=work)
    _sync()
    for (k, rule, steps, sid), init, (_, _, _, _, b0, b1) in zip(specs, inits, inst):
        got = b0 if steps % 2 == 0 else b1
        ref = _alone(k, rule, steps, init)
        _sync()
        assert torch.equal(got.view(torch.uint8), ref.view(torch.uint8)), (k, rule, steps)
        if k <= 9:
            want = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), steps)
            assert_match(k, rule, got.cpu().numpy(), want, f"batch k={k} rule={rule}")


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_level8_to_13_many_steps(persistent):
    """64 gaskets of levels 8..13, half automaton half heat, 120 steps each
    (the structure of the 256-gasket batch at a size a test can afford)."""
    torch = torch_dev()
    pairs = fi.batch_instances(64, 2004, 8, 13)
    inst, alone = [], []
    for j, (k, rule) in enumerate(pairs):
        b0, b1 = zeros_state(k, rule), zeros_state(k, rule)
        F.seed_fill(k, rule, 50 + j, b0)
        inst.append((k, rule, 120, ALPHA, b0, b1))
    F.batch_step(inst, tuning=(F.R_AUTO, 0, 0, F.FLAG_PERSISTENT) if persistent else None)
    _sync()
    for j, (k, rule) in enumerate(pairs):
        a0, a1 = zeros_state(k, rule), zeros_state(k, rule)
        F.seed_fill(k, rule, 50 + j, a0)
        F.lambda_step(k, F.R_AUTO, rule, ALPHA, a0, a1, 120)
        _sync()
        assert torch.equal(inst[j][4].view(torch.uint8), a0.view(torch.uint8)), (j, k, rule)
        del a0, a1


def test_batch_workspace_size_and_short_workspace():
    """The workspace holds the per-instance offset table (6 entries of 48
    bytes per instance, rounded to 256 bytes); a short one is refused before
    anything is enqueued."""
    torch = torch_dev()
    assert F.batch_workspace(0) == 0
    assert F.batch_workspace(1) == 512
    assert F.batch_workspace(40) == (40 * 6 * 48 + 255) // 256 * 256
    k, rule = 6, fi.RULE_CA
    init = fi.window_values(k, rule, 2)
    b0, b1 = to_device(init), zeros_state(k, rule)
    short = torch.empty(128, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FractalError) as e:
        F.batch_step([(k, rule, 3, ALPHA, b0, b1)], work=short)
    assert e.value.code == F.E_INVAL
    _sync()
    assert torch.equal(b0.cpu(), torch.from_numpy(init)), "a refused call changed the state"


def test_batch_repeated_calls_reuse_state():
    """Two batch calls in a row continue from the first call's result."""
    torch = torch_dev()
    k, rule = 9, fi.RULE_HEAT
    init = fi.window_values(k, rule, 4)
    b0, b1 = to_device(init), zeros_state(k, rule)
    F.batch_step([(k, rule, 6, ALPHA, b0, b1)])
    F.batch_step([(k, rule, 5, ALPHA, b0, b1)])
    _sync()
    ref = _alone(k, rule, 11, init)
    _sync()
    assert torch.equal(b1.view(torch.uint8), ref.view(torch.uint8))


def _arena(gib):
    torch = torch_dev()
    nbytes = int(gib * (1 << 30))
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda"), nbytes


def _wait(srv, tickets, timeout=120.0):
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.001)
    return out


def _checksum(arr):
    if arr.dtype == np.uint8:
        return int(arr.astype(np.uint64).sum()) % (1 << 64)
    return int(arr.view(np.uint32).astype(np.uint64).sum()) % (1 << 64)


def test_serve_alone_equals_in_mix():
    torch = torch_dev()
    arena, nbytes = _arena(2)
    specs = _mix(24, 11, 2, 11, 60)
    with F.Server(arena, nbytes, max_slots=8, steps_per_iter=7) as srv:
        tickets, outs = [], []
        for (k, rule, steps, sid) in specs:
            n = 1 << k
            out = np.zeros((n, n), dtype=np.uint8 if rule == 0 else np.float32)
            outs.append(out)
            tickets.append(srv.submit(k, rule, steps, ALPHA, seed=sid, h_out=out))
        res = _wait(srv, tickets)
    for t, (k, rule, steps, sid), out in zip(tickets, specs, outs):
        status, ta, tad, td, csum = res[t]
        assert status == 0 and ta <= tad <= td
        init = fi.window_values(k, rule, sid)
        ref = _alone(k, rule, steps, init)
        _sync()
        assert np.array_equal(out.view(np.uint8), ref.cpu().numpy().view(np.uint8)), (k, rule, steps)
        assert csum == _checksum(out)
        if k <= 8:
            want = oracle_steps(k, rule, init if rule == 0 else init.astype(np.float64), steps)
            assert_match(k, rule, out, want, f"serve k={k}")
    del torch


def test_serve_fifo_under_memory_pressure_and_host_init():
    """An arena that holds about two level-11 float32 requests: the rest
    wait their turn, are admitted first come first served, and finish with
    correct results (initial state uploaded from host memory)."""
    torch = torch_dev()
    k, rule = 11, fi.RULE_HEAT
    need = 2 * (1 << (2 * k)) * 4
    arena, _ = _arena(0.08)
    nbytes = int(2.3 * need) + (1 << 20)
    with F.Server(arena, nbytes, max_slots=8, steps_per_iter=4) as srv:
        tickets, outs, inits = [], [], []
        for j in range(6):
            init = fi.window_values(k, rule, 300 + j)
            out = np.zeros_like(init)
            inits.append(init)
            outs.append(out)
            tickets.append(srv.submit(k, rule, 10 + j, ALPHA, h_init=init, h_out=out))
        res = _wait(srv, tickets)
    admits = [res[t][2] for t in tickets]
    assert admits == sorted(admits), "admission not first come first served"
    for j, t in enumerate(tickets):
        assert res[t][0] == 0
        want = oracle_steps(k, rule, inits[j].astype(np.float64), 10 + j)
        assert_match(k, rule, outs[j], want, f"request {j}")
    del torch


def test_serve_rejections():
    arena, nbytes = _arena(0.01)
    with F.Server(arena, nbytes, max_slots=2) as srv:
        for bad in (0, -3):
            with pytest.raises(F.FractalError) as e:
                srv.set_steps_per_iter(bad)
            assert e.value.code == F.E_INVAL
        srv.set_steps_per_iter(5)
        with pytest.raises(F.FractalError) as e:
            srv.submit(14, 1, 5)  # 2 GiB footprint > 10 MiB arena
        assert e.value.code == F.E_NOMEM
        with pytest.raises(F.FractalError) as e:
            srv.submit(5, 1, 5, alpha=0.5)
        assert e.value.code == F.E_INVAL
        with pytest.raises(F.FractalError) as e:
            srv.poll(987654)
        assert e.value.code == F.E_INVAL
        t = srv.submit(6, 0, 0, seed=3)  # zero steps: the seeded state itself
        res = _wait(srv, [t])[t]
        init = fi.window_values(6, 0, 3)
        assert res[0] == 0 and res[4] == _checksum(init)
