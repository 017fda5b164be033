"""The allocation-free reduction (fractal_reduce_noalloc) against
fractal_reduce with a caller workspace: the same result, bit for bit, on two
calls in a row (the second smaller, so stale scratch from the first would
show), on both maps and both cell types, at the largest block level the
static scratch holds; larger block levels are refused before any device
work."""
import numpy as np
import pytest

import fractal_inputs as fi
import oracle
import paper_2004_13475_amd as F

from gpu_util import torch_dev

RULES = [fi.RULE_CA, fi.RULE_HEAT]


def test_noalloc_refuses_block_levels_beyond_scratch():
    """k - r = 14 needs 38 MB of slots, beyond the 16 MiB scratch: E_INVAL,
    decided on the host (no device is touched)."""
    F.load()
    with pytest.raises(F.FractalError) as e:
        F.reduce_noalloc(F.MAP_LAMBDA, 16, 2, F.RULE_CA, 1 << 20, 1 << 21, stream=0)
    assert e.value.code == F.E_INVAL and "fractal_reduce" in str(e.value)
    with pytest.raises(F.FractalError) as e:  # misaligned output
        F.reduce_noalloc(F.MAP_LAMBDA, 10, 4, F.RULE_CA, 1 << 20, (1 << 21) + 4, stream=0)
    assert e.value.code == F.E_INVAL


def _both(map_, k, r, rule, buf, torch):
    """(workspace result, scratch result) as raw 8-byte words."""
    work = torch.empty(max(8, F.reduce_workspace(k, r)), dtype=torch.uint8, device="cuda")
    want = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    got = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    F.reduce(map_, k, r, rule, buf, work, want)
    F.reduce_noalloc(map_, k, r, rule, buf, got)
    torch.cuda.synchronize()
    return int(want.item()), int(got.item())


@pytest.mark.gpu
@pytest.mark.parametrize("rule", RULES)
def test_noalloc_equals_workspace_reduce(rule):
    torch = torch_dev()
    for map_ in (F.MAP_LAMBDA, F.MAP_BB):
        # a larger call, then a smaller one on the same scratch, then the
        # largest block level the scratch holds (k - r = 13)
        for (k, r, seed) in ((12, 4, 31), (8, 3, 32), (16, 3, 33)):
            n = 1 << k
            dt = torch.uint8 if rule == fi.RULE_CA else torch.float32
            buf = torch.empty((n, n), dtype=dt, device="cuda")
            F.seed_fill(k, rule, seed, buf)
            want, got = _both(map_, k, r, rule, buf, torch)
            assert got == want, (map_, k, r, want, got)
            if k <= 12:
                # and the oracle's exact sum (seeded values are exact in
                # float64 sums: uint8, or multiples of 2^-24 below 1)
                st = fi.full_state(k, rule, seed)
                ref = oracle.reduce_(k, st)
                if rule == fi.RULE_CA:
                    assert got == int(ref), (k, r, got, ref)
                else:
                    val = np.array([got], dtype=np.int64).view(np.float64)[0]
                    assert val == float(ref), (k, r, val, ref)
            del buf
            torch.cuda.empty_cache()
