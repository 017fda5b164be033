"""Helpers for the GPU parity tests: device buffers via torch, the heat error
metric, and the oracle's light-cone windows for sampled full-size checks."""
from __future__ import annotations

import numpy as np

import fractal_inputs as fi
import oracle

ALPHA = float(np.float32(0.2))   # the float32 coefficient, exactly, in float64
HEAT_TOL = 1e-5
TINY = 2.0 ** -126               # smallest normal float32


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a visible device"
    return torch


def dtype_of(rule):
    torch = torch_dev()
    return torch.uint8 if rule == fi.RULE_CA else torch.float32


def to_device(arr: np.ndarray):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda")


def zeros_state(k, rule):
    torch = torch_dev()
    n = 1 << k
    return torch.zeros((n, n), dtype=dtype_of(rule), device="cuda")


def heat_err(gpu: np.ndarray, ref: np.ndarray) -> float:
    """max |g - r| / max(|r|, 2^-126): relative error, with the smallest
    normal float32 as the floor once the reference decays below it."""
    g = gpu.astype(np.float64)
    if g.size == 0:
        return 0.0
    return float(np.max(np.abs(g - ref) / np.maximum(np.abs(ref), TINY)))


def oracle_steps(k, rule, state, steps, x0=0, y0=0):
    if rule == fi.RULE_CA:
        return oracle.ca_run(k, state, steps, x0, y0)
    return oracle.heat_run(k, state.astype(np.float64), ALPHA, steps, x0, y0)


def assert_match(k, rule, gpu: np.ndarray, ref: np.ndarray, what=""):
    if rule == fi.RULE_CA:
        bad = np.argwhere(gpu != ref)
        assert bad.size == 0, f"{what}: {len(bad)} cells differ, first {bad[:5].tolist()}"
    else:
        e = heat_err(gpu, ref)
        assert e <= HEAT_TOL, f"{what}: heat error {e:.3e} > {HEAT_TOL}"


def window_plan(k, steps, out_w, out_h, cx, cy):
    """Window whose valid interior after `steps` steps covers the output box
    [cx, cx+out_w) x [cy, cy+out_h) (clipped to the array)."""
    n = 1 << k
    x0 = max(0, cx - steps)
    y0 = max(0, cy - steps)
    x1 = min(n, cx + out_w + steps)
    y1 = min(n, cy + out_h + steps)
    return x0, y0, x1 - x0, y1 - y0
