"""Seeded synthetic inputs for the Sierpinski-gasket stencil workloads.

This module is shared by the tests, the benchmark and the CPU oracle's callers.
It holds no arithmetic of the method (no block map, no stencil): only the
counter-based random generator and the domain predicate that says which cells of
the n x n embedding belong to the gasket.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the 64-bit finaliser constants are Vigna's).
Cell (x, y) of an instance with 32-bit stream id `stream` in an n x n embedding
takes counter i = stream * 2**32 + (y * n + x) and draws
    z = mix64((i + 1) * GAMMA mod 2**64),
i.e. output number i + 1 of a SplitMix64 generator started from state 0.
The GPU library implements the same published definition independently
(its seeded fill entry point); tests check the two bit for bit.

Values:
  rule 0 (cellular automaton, uint8): member ? z >> 63 : 0   (Bernoulli(1/2))
  rule 1 (heat, float32):             member ? (z >> 40) * 2**-24 : 0
                                       (U[0,1) on a 24-bit grid, exact in
                                        float32 and float64)
A cell is a member of the level-k gasket iff (x & y) == 0.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

RULE_CA = 0
RULE_HEAT = 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_counter(i: np.ndarray) -> np.ndarray:
    """Output number i+1 of SplitMix64 started from state 0."""
    i = np.asarray(i, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64((i + np.uint64(1)) * GAMMA)


def member_mask(k: int, x0: int = 0, y0: int = 0, w: int | None = None,
                h: int | None = None) -> np.ndarray:
    """Boolean (h, w) array: True where (x & y) == 0 for the window cells."""
    n = 1 << k
    w = n if w is None else w
    h = n if h is None else h
    xs = np.arange(x0, x0 + w, dtype=np.int64)
    ys = np.arange(y0, y0 + h, dtype=np.int64)
    inside = ((xs >= 0) & (xs < n))[None, :] & ((ys >= 0) & (ys < n))[:, None]
    return inside & ((ys[:, None] & xs[None, :]) == 0)


def window_values(k: int, rule: int, stream: int, x0: int = 0, y0: int = 0,
                  w: int | None = None, h: int | None = None,
                  dtype=None) -> np.ndarray:
    """Seeded initial state of the window [x0, x0+w) x [y0, y0+h).

    Cells outside [0, n)^2 or off the gasket are 0.  Returns uint8 for the
    automaton and float32 for heat (float64 if dtype=np.float64; the values
    are exact in both).
    """
    n = 1 << k
    w = n if w is None else w
    h = n if h is None else h
    xs = np.arange(x0, x0 + w, dtype=np.int64)
    ys = np.arange(y0, y0 + h, dtype=np.int64)
    mem = member_mask(k, x0, y0, w, h)
    xc = np.clip(xs, 0, n - 1).astype(np.uint64)
    yc = np.clip(ys, 0, n - 1).astype(np.uint64)
    base = np.uint64(stream & 0xFFFFFFFF) << np.uint64(32)
    idx = base + yc[:, None] * np.uint64(n) + xc[None, :]
    z = splitmix64_counter(idx)
    if rule == RULE_CA:
        out = (z >> np.uint64(63)).astype(np.uint8)
        out[~mem] = 0
        return out
    if rule == RULE_HEAT:
        v = (z >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)
        v[~mem] = 0.0
        return v.astype(dtype if dtype is not None else np.float32)
    raise ValueError(f"unknown rule {rule}")


def full_state(k: int, rule: int, stream: int, dtype=None) -> np.ndarray:
    """Whole n x n seeded state (row-major, cell (x, y) at [y, x])."""
    n = 1 << k
    if n <= 2048:
        return window_values(k, rule, stream, dtype=dtype)
    rows = []
    step = max(1, (1 << 22) // n)
    for y in range(0, n, step):
        rows.append(window_values(k, rule, stream, 0, y, n, min(step, n - y),
                                  dtype=dtype))
    return np.concatenate(rows, axis=0)


def batch_instances(count: int, seed: int, kmin: int, kmax: int):
    """Seeded list of (k, rule) pairs for a batch of gaskets.

    Levels are uniform in [kmin, kmax]; the first half of a seeded permutation
    runs the automaton and the rest heat.  Uses numpy's PCG64 with `seed`.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = rng.integers(kmin, kmax + 1, size=count)
    perm = rng.permutation(count)
    rules = np.empty(count, dtype=np.int64)
    rules[perm[: count // 2]] = RULE_CA
    rules[perm[count // 2:]] = RULE_HEAT
    return [(int(a), int(b)) for a, b in zip(ks, rules)]
