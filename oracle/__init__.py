"""Python face of the plain CPU oracle (``fractal_oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library and never imports it.

Functions mirror the C file one to one; each docstring names the passage of
the paper it follows.  Parity status: every function below is pinned by
``tests/test_oracle_pins.py`` (closed forms, brute force, a textbook-routine
special case, hand-derived values); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fractal_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

RULE_CA = 0
RULE_HEAT = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE doubles)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    vp = ctypes.c_void_p
    lib.oracle_member.argtypes = [i64, i64, i32]
    lib.oracle_member.restype = i32
    lib.oracle_count_members.argtypes = [i32]
    lib.oracle_count_members.restype = u64
    lib.oracle_grid_dims.argtypes = [i32, ctypes.POINTER(u64),
                                     ctypes.POINTER(u64)]
    lib.oracle_grid_dims.restype = None
    lib.oracle_lambda_paper.argtypes = [i32, u64, u64, ctypes.POINTER(u64),
                                        ctypes.POINTER(u64)]
    lib.oracle_lambda.argtypes = lib.oracle_lambda_paper.argtypes
    lib.oracle_lambda_grid.argtypes = [i32, i32, vp]
    lib.oracle_nonempty_blocks.argtypes = [i32, i32, vp]
    lib.oracle_ca_run.argtypes = [i32, i64, i64, i64, i64, vp, i32, vp]
    lib.oracle_ca_run.restype = i32
    lib.oracle_heat_run.argtypes = [i32, i64, i64, i64, i64, vp,
                                    ctypes.c_double, i32, vp]
    lib.oracle_heat_run.restype = i32
    lib.oracle_threads.restype = i32
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads the oracle's steppers use."""
    return _load().oracle_threads()


def member(x: int, y: int, k: int) -> bool:
    """Gasket membership, (x & y) == 0 inside [0, 2^k)^2 (Section 6.1 test,
    mirrored)."""
    return bool(_load().oracle_member(x, y, k))


def count_members(k: int) -> int:
    """Brute-force member count of the level-k gasket (Eq. 2 says 3^k)."""
    return int(_load().oracle_count_members(k))


def grid_dims(rb: int):
    """Compact grid 3^ceil(rb/2) x 3^floor(rb/2) (Lemma 2)."""
    gx, gy = ctypes.c_uint64(), ctypes.c_uint64()
    _load().oracle_grid_dims(rb, ctypes.byref(gx), ctypes.byref(gy))
    return int(gx.value), int(gy.value)


def lambda_paper(rb: int, wx: int, wy: int):
    """lambda(omega) in the paper's orientation (Theorem 1, Section 6.1)."""
    lx, ly = ctypes.c_uint64(), ctypes.c_uint64()
    _load().oracle_lambda_paper(rb, wx, wy, ctypes.byref(lx), ctypes.byref(ly))
    return int(lx.value), int(ly.value)


def lambda_(rb: int, wx: int, wy: int):
    """lambda(omega) for the (x & y) == 0 embedding (paper's value mirrored)."""
    lx, ly = ctypes.c_uint64(), ctypes.c_uint64()
    _load().oracle_lambda(rb, wx, wy, ctypes.byref(lx), ctypes.byref(ly))
    return int(lx.value), int(ly.value)


def lambda_grid(rb: int, paper_orient: bool = False) -> np.ndarray:
    """lambda over the whole compact grid: array (gy, gx, 2) uint32,
    [wy, wx] = (lambda_x, lambda_y)."""
    gx, gy = grid_dims(rb)
    out = np.zeros((gy, gx, 2), dtype=np.uint32)
    _load().oracle_lambda_grid(rb, int(paper_orient), out.ctypes.data)
    return out


def nonempty_blocks(k: int, r: int) -> np.ndarray:
    """(n_b, n_b) uint8 mask of blocks holding a member, by scanning cells
    (what the bounding-box approach discards: Section 1, Section 6.2)."""
    nb = 1 << (k - r)
    out = np.zeros((nb, nb), dtype=np.uint8)
    _load().oracle_nonempty_blocks(k, r, out.ctypes.data)
    return out


def ca_run(k: int, state: np.ndarray, steps: int, x0: int = 0,
           y0: int = 0) -> np.ndarray:
    """`steps` automaton steps (Section 6.2 test CA, rule B3/S23) on the
    window whose top-left cell is (x0, y0); `state` is (h, w) uint8."""
    a = np.ascontiguousarray(state, dtype=np.uint8)
    h, w = a.shape
    out = np.empty_like(a)
    rc = _load().oracle_ca_run(k, x0, y0, w, h, a.ctypes.data, steps,
                               out.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_ca_run: out of memory")
    return out


def heat_run(k: int, state: np.ndarray, alpha: float, steps: int,
             x0: int = 0, y0: int = 0) -> np.ndarray:
    """`steps` float64 heat steps (5-point, Dirichlet 0 off the gasket) on the
    window whose top-left cell is (x0, y0)."""
    a = np.ascontiguousarray(state, dtype=np.float64)
    h, w = a.shape
    out = np.empty_like(a)
    rc = _load().oracle_heat_run(k, x0, y0, w, h, a.ctypes.data,
                                 float(alpha), steps, out.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_heat_run: out of memory")
    return out


def valid_interior(k: int, x0: int, y0: int, w: int, h: int, steps: int):
    """Slices (rows, cols) of a window result that are exact after `steps`
    steps: cells within `steps` of a window edge that is not an array edge
    may have seen the zeros assumed outside the window."""
    n = 1 << k
    lo_x = 0 if x0 <= 0 else steps
    lo_y = 0 if y0 <= 0 else steps
    hi_x = w if x0 + w >= n else w - steps
    hi_y = h if y0 + h >= n else h - steps
    return slice(lo_y, max(lo_y, hi_y)), slice(lo_x, max(lo_x, hi_x))


def gasket_mask(k: int) -> np.ndarray:
    """Membership of every cell of the n x n embedding (Eq. 2 set): cell
    (x, y) belongs to the level-k gasket iff x & y == 0.  Row y, column x."""
    n = 1 << k
    ax = np.arange(n, dtype=np.int64)
    return np.bitwise_and.outer(ax, ax) == 0


def single_write(k: int, rule: int, value: int) -> np.ndarray:
    """Section 6.2, test SW: a constant written on every element of the
    gasket, embedded in an n x n array that starts at 0.  `value` is the low
    byte for the automaton's uint8 cells, the float32 bit pattern for heat
    cells."""
    mask = gasket_mask(k)
    if rule == 0:
        out = np.zeros(mask.shape, dtype=np.uint8)
        out[mask] = value & 0xFF
    else:
        out = np.zeros(mask.shape, dtype=np.float32)
        out[mask] = np.array([value & 0xFFFFFFFF], dtype=np.uint32).view(np.float32)[0]
    return out


def reduce_(k: int, state: np.ndarray):
    """Section 6.2, test RD: the arithmetic sum of all elements of the
    gasket (cells off the gasket do not take part).  uint8 states give the
    exact integer; float states give the exactly rounded float64 sum
    (math.fsum)."""
    vals = np.asarray(state)[gasket_mask(k)]
    if vals.dtype == np.uint8:
        return int(vals.astype(np.int64).sum())
    return math.fsum(vals.astype(np.float64).tolist())


def compact_index(k: int, r: int, x, y):
    """Offset of cell (x, y) in compact storage (Section 7: the data packed
    into the orthotope by lambda^-1): tiles of side 2^r kept in the order
    whose base-3 digits beta_mu (mu = 1..k-r) give the tile's block through
    Theorem 1's table (mirrored: x bit = [beta == 2], y bit = [beta == 0]),
    each tile's box row-major.  Inverting digit by digit: beta_mu = 2 where
    bit mu-1 of the block x is set, 0 where that of y is, 1 where neither.
    Works on integers or integer arrays."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    rho = 1 << r
    bx, by = x >> r, y >> r
    L = np.zeros_like(x)
    for mu in range(k - r - 1, -1, -1):
        xb = (bx >> mu) & 1
        yb = (by >> mu) & 1
        L = 3 * L + np.where(xb == 1, 2, np.where(yb == 1, 0, 1))
    return (L * rho + (y & (rho - 1))) * rho + (x & (rho - 1))


def pack(k: int, r: int, state: np.ndarray) -> np.ndarray:
    """The compact state (1-D, 3^(k-r) * 4^r cells) holding the boxes of the
    non-empty tiles of the n x n `state`."""
    n = 1 << k
    rho = 1 << r
    out = np.zeros(3 ** (k - r) * rho * rho, dtype=state.dtype)
    ys, xs = np.meshgrid(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64),
                         indexing="ij")
    live = ((xs >> r) & (ys >> r)) == 0
    out[compact_index(k, r, xs[live], ys[live])] = state[live]
    return out


def unpack(k: int, r: int, compact: np.ndarray) -> np.ndarray:
    """The n x n state whose non-empty tile boxes come from `compact` (cells
    of empty tiles 0)."""
    n = 1 << k
    out = np.zeros((n, n), dtype=compact.dtype)
    ys, xs = np.meshgrid(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64),
                         indexing="ij")
    live = ((xs >> r) & (ys >> r)) == 0
    out[live] = compact[compact_index(k, r, xs[live], ys[live])]
    return out


# ------------------------------------------------------------ NBB family
def nbb_member_mask(replicas, s: int, level: int, x0: int = 0, y0: int = 0,
                    w: int | None = None, h: int | None = None) -> np.ndarray:
    """Membership of the level-`level` NBB fractal (Section 3): cell (x, y)
    of the s^level x s^level embedding belongs to it iff, at every scale, the
    base-s digit pair (x_d, y_d) is the offset of one of the replicas.  For
    the window [x0, x0+w) x [y0, y0+h); cells outside the embedding are not
    members."""
    n = s ** level
    w = n if w is None else w
    h = n if h is None else h
    xs = np.arange(x0, x0 + w, dtype=np.int64)[None, :]
    ys = np.arange(y0, y0 + h, dtype=np.int64)[:, None]
    allowed = np.zeros((s, s), dtype=bool)
    for (tx, ty) in replicas:
        allowed[ty, tx] = True
    m = (xs >= 0) & (xs < n) & (ys >= 0) & (ys < n)
    xv, yv = np.clip(xs, 0, n - 1), np.clip(ys, 0, n - 1)
    for _ in range(level):
        m = m & allowed[yv % s, xv % s]
        xv, yv = xv // s, yv // s
    return m


def nbb_lambda(replicas, s: int, rb: int, wx: int, wy: int):
    """Theorem 1 for any NBB table, step by step: for mu = 1..rb, beta_mu is
    the base-k digit ceil(mu/2) - 1 of omega_x (odd mu) or omega_y (even
    mu), tau = H[beta_mu], Delta^mu = tau * s^(mu-1), and lambda is the sum
    of the Delta^mu."""
    k = len(replicas)
    lx = ly = 0
    for mu in range(1, rb + 1):
        v = wx if mu % 2 == 1 else wy
        beta = (v // k ** ((mu + 1) // 2 - 1)) % k
        tx, ty = replicas[beta]
        lx += tx * s ** (mu - 1)
        ly += ty * s ** (mu - 1)
    return lx, ly


def nbb_single_write(replicas, s: int, level: int, value: int) -> np.ndarray:
    """Test SW on an NBB fractal: `value` (uint8) on every member, 0 elsewhere."""
    return nbb_member_mask(replicas, s, level).astype(np.uint8) * np.uint8(value & 0xFF)


def nbb_reduce(replicas, s: int, level: int, state: np.ndarray) -> int:
    """Test RD on an NBB fractal: the exact integer sum of the members."""
    return int(np.asarray(state)[nbb_member_mask(replicas, s, level)].astype(np.int64).sum())


def nbb_ca_run(replicas, s: int, level: int, state: np.ndarray, steps: int,
               x0: int = 0, y0: int = 0) -> np.ndarray:
    """`steps` synchronous steps of the test-CA rule (Section 6.2: Moore
    neighbourhood, fractal cells only, B3/S23) on a window of the NBB
    fractal whose top-left cell is (x0, y0); cells outside the window count
    as dead."""
    a = (np.asarray(state) != 0).astype(np.int64)
    h, w = a.shape
    mask = nbb_member_mask(replicas, s, level, x0, y0, w, h)
    a = a * mask
    for _ in range(steps):
        p = np.pad(a, 1)
        cnt = sum(p[1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
                  for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy) != (0, 0))
        a = (((cnt == 3) | ((a == 1) & (cnt == 2))) & mask).astype(np.int64)
    return a.astype(np.uint8)
