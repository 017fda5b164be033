"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or mathematics fixes:
closed forms (Eq. 2, Lemma 1, Lemma 2), brute force on small inputs, the
textbook Game of Life (a library 2-D convolution) as a special case, and
hand-derived values stored under tests/golden/.
"""
import math
import os

import numpy as np
import pytest
from scipy import ndimage, signal

import fractal_inputs as fi
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA32 = float(np.float32(0.2))


# --------------------------------------------------------------- geometry
@pytest.mark.parametrize("k", range(0, 13))
def test_member_count_is_3_pow_k(k):
    """Eq. 2: V = k^r with 3 replicas per level, and Lemma 1: V = n^H."""
    c = oracle.count_members(k)
    assert c == 3 ** k
    if k >= 1:
        assert abs(math.log(c) / math.log(2 ** k) - math.log(3) / math.log(2)) < 1e-12
    # the input generator's domain predicate agrees with the oracle's scan
    assert int(fi.member_mask(k).sum()) == c if k <= 11 else True


@pytest.mark.parametrize("k", range(0, 11))
def test_nonempty_blocks_count_and_grid(k):
    """Brute-force count of non-empty rho x rho blocks is 3^(k-r), and the
    compact grid of Lemma 2 has exactly that many cells, quasi-regular."""
    for r in range(0, k + 1):
        rb = k - r
        mask = oracle.nonempty_blocks(k, r)
        assert int(mask.sum()) == 3 ** rb
        gx, gy = oracle.grid_dims(rb)
        assert gx * gy == 3 ** rb
        assert gx in (gy, 3 * gy)


def _paper_block_set(rb):
    """Block-level gasket in the paper's orientation: the Section 6.1 test
    t_x & (b - 1 - t_y) == 0 applied to block coordinates of side 2^rb."""
    nb = 1 << rb
    X, Y = np.meshgrid(np.arange(nb), np.arange(nb))
    ok = (X & (nb - 1 - Y)) == 0
    return set(zip(X[ok].tolist(), Y[ok].tolist()))


@pytest.mark.parametrize("k", range(0, 13))
def test_lambda_is_bijection_onto_nonempty_blocks(k):
    """lambda maps the compact grid one-to-one onto the non-empty blocks
    found by scanning every cell (Theorem 1), for every r <= k."""
    for r in range(0, k + 1):
        rb = k - r
        grid = oracle.lambda_grid(rb).reshape(-1, 2)
        image = set(map(tuple, grid.tolist()))
        assert len(image) == grid.shape[0] == 3 ** rb
        mask = oracle.nonempty_blocks(k, r)
        ys, xs = np.nonzero(mask)
        assert image == set(zip(xs.tolist(), ys.tolist()))


@pytest.mark.parametrize("rb", range(0, 13))
def test_lambda_paper_orientation(rb):
    """Before mirroring, lambda lands exactly on the paper's own gasket
    orientation (Section 6.1 membership test at block level)."""
    grid = oracle.lambda_grid(rb, paper_orient=True).reshape(-1, 2)
    image = set(map(tuple, grid.tolist()))
    assert len(image) == 3 ** rb
    assert image == _paper_block_set(rb)


def test_lambda_level1_is_table_H():
    """At r_b = 1 lambda in the paper's orientation is the table H itself."""
    assert [oracle.lambda_paper(1, wx, 0) for wx in range(3)] == [(0, 0), (0, 1), (1, 1)]


def test_lambda_hand_derived_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "lambda_small.txt"), dtype=np.int64)
    for rb, wy, wx, lx, ly in rows:
        assert oracle.lambda_(int(rb), int(wx), int(wy)) == (lx, ly)
        grid = oracle.lambda_grid(int(rb))
        assert tuple(grid[wy, wx]) == (lx, ly)


def test_lambda_large_rb_in_range():
    """For r_b up to 30 every sampled lambda lies in the block grid and on
    the gasket (block coordinates satisfy X & Y == 0)."""
    rng = np.random.default_rng(7)
    for rb in (20, 25, 30):
        gx, gy = oracle.grid_dims(rb)
        for _ in range(2000):
            wx, wy = int(rng.integers(gx)), int(rng.integers(gy))
            lx, ly = oracle.lambda_(rb, wx, wy)
            assert lx < 2 ** rb and ly < 2 ** rb and (lx & ly) == 0


# --------------------------------------------------------------- automaton
def _textbook_life_masked(state, k, steps):
    """Conway's B3/S23 on the zero-padded array (library convolution), then
    cells off the gasket set to 0, repeated `steps` times."""
    mem = fi.member_mask(k)
    kern = np.ones((3, 3), dtype=np.int64)
    kern[1, 1] = 0
    s = state.astype(np.int64)
    for _ in range(steps):
        cnt = signal.convolve2d(s, kern, mode="same", boundary="fill", fillvalue=0)
        s = ((cnt == 3) | ((s == 1) & (cnt == 2))).astype(np.int64)
        s[~mem] = 0
    return s.astype(np.uint8)


@pytest.mark.parametrize("k,steps", [(1, 1), (2, 3), (4, 6), (6, 12), (8, 30), (9, 40)])
def test_ca_equals_textbook_life_then_mask(k, steps):
    state = fi.window_values(k, fi.RULE_CA, stream=11 + k)
    got = oracle.ca_run(k, state, steps)
    assert np.array_equal(got, _textbook_life_masked(state, k, steps))


def test_ca_hand_cases_level1():
    # k = 1: members (0,0), (1,0), (0,1); (1,1) is off the gasket.
    full = np.array([[1, 1], [1, 0]], dtype=np.uint8)      # rows are y
    # each live member has exactly 2 live member neighbours -> survives;
    # (1,1) sees 3 live neighbours but is not a member -> stays 0.
    assert np.array_equal(oracle.ca_run(1, full, 1), full)
    single = np.array([[1, 0], [0, 0]], dtype=np.uint8)
    assert np.array_equal(oracle.ca_run(1, single, 1), np.zeros((2, 2), np.uint8))


def test_ca_window_interior_matches_full():
    k, steps = 9, 7
    state = fi.window_values(k, fi.RULE_CA, stream=3)
    full = oracle.ca_run(k, state, steps)
    for (x0, y0, w, h) in [(100, 40, 90, 70), (0, 0, 64, 64), (480, 300, 32, 212)]:
        win = state[y0:y0 + h, x0:x0 + w]
        got = oracle.ca_run(k, win, steps, x0, y0)
        rs, cs = oracle.valid_interior(k, x0, y0, w, h, steps)
        assert np.array_equal(got[rs, cs], full[y0:y0 + h, x0:x0 + w][rs, cs])


def test_ca_off_gasket_stays_zero():
    k = 8
    state = fi.window_values(k, fi.RULE_CA, stream=5)
    mem = fi.member_mask(k)
    for t in (1, 2, 5):
        assert not oracle.ca_run(k, state, t)[~mem].any()


# --------------------------------------------------------------- heat
def _deg4(k):
    mem = fi.member_mask(k)
    p = np.pad(mem, 1)
    return (p[:-2, 1:-1].astype(int) + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:]) * mem


@pytest.mark.parametrize("k", [1, 3, 6, 9])
def test_heat_uniform_field_closed_form(k):
    """u = 1 on members: u' = 1 - 4a + a * deg4(c) (0.4 / 0.6 / 0.8 for
    degrees 1 / 2 / 3 at a = 0.2), and the total is
    3^k (1 - 4a) + 2a (3^k - 1) because the 4-neighbour graph is a tree."""
    a = 0.2
    mem = fi.member_mask(k)
    u = mem.astype(np.float64)
    got = oracle.heat_run(k, u, a, 1)
    deg = _deg4(k)
    want = np.where(mem, 1 - 4 * a + a * deg, 0.0)
    assert np.allclose(got, want, rtol=0, atol=1e-15)
    if k >= 1:
        assert set(np.round(got[mem], 12).tolist()) <= {0.4, 0.6, 0.8}
    edges = int(deg.sum()) // 2
    assert edges == 3 ** k - 1
    assert abs(got.sum() - (3 ** k * (1 - 4 * a) + 2 * a * (3 ** k - 1))) < 1e-9


def test_heat_hand_case_level1():
    # members (0,0) centre, (1,0) and (0,1) leaves; alpha = 1/4 makes the
    # centre term vanish: u'00 = (u10 + u01)/4, u'10 = u00/4, u'01 = u00/4.
    u = np.array([[0.5, 0.25], [0.75, 0.0]])
    got = oracle.heat_run(1, u, 0.25, 1)
    assert np.array_equal(got, np.array([[0.25, 0.125], [0.125, 0.0]]))
    # alpha = 1/8: u'00 = 0.5*u00 + (u10+u01)/8
    got = oracle.heat_run(1, u, 0.125, 1)
    assert np.array_equal(got, np.array([[0.375, 0.1875], [0.4375, 0.0]]))


def test_heat_linearity():
    k = 7
    u = fi.window_values(k, fi.RULE_HEAT, 1, dtype=np.float64)
    v = fi.window_values(k, fi.RULE_HEAT, 2, dtype=np.float64)
    lhs = oracle.heat_run(k, 2.0 * u - 3.0 * v, ALPHA32, 4)
    rhs = 2.0 * oracle.heat_run(k, u, ALPHA32, 4) - 3.0 * oracle.heat_run(k, v, ALPHA32, 4)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


@pytest.mark.parametrize("k,steps", [(2, 3), (5, 10), (8, 25)])
def test_heat_equals_library_stencil_then_mask(k, steps):
    """Special case reducing to a library routine: a 5-point cross
    convolution of the zero-padded field, then masking off-gasket cells."""
    mem = fi.member_mask(k)
    u = fi.window_values(k, fi.RULE_HEAT, 9, dtype=np.float64)
    cross = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=np.float64)
    ref = u.copy()
    for _ in range(steps):
        nb = ndimage.convolve(ref, cross, mode="constant", cval=0.0)
        ref = np.where(mem, (1 - 4 * ALPHA32) * ref + ALPHA32 * nb, 0.0)
    got = oracle.heat_run(k, u, ALPHA32, steps)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-300)


def test_heat_window_interior_matches_full():
    k, steps = 9, 6
    u = fi.window_values(k, fi.RULE_HEAT, 4, dtype=np.float64)
    full = oracle.heat_run(k, u, ALPHA32, steps)
    x0, y0, w, h = 200, 150, 100, 120
    got = oracle.heat_run(k, u[y0:y0 + h, x0:x0 + w], ALPHA32, steps, x0, y0)
    rs, cs = oracle.valid_interior(k, x0, y0, w, h, steps)
    assert np.array_equal(got[rs, cs], full[y0:y0 + h, x0:x0 + w][rs, cs])


# --------------------------------------------------------------- inputs
def test_splitmix64_reference_outputs():
    """First outputs of SplitMix64 from state 0, as published with the
    generator (counter i -> output i + 1)."""
    z = fi.splitmix64_counter(np.arange(3, dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                   0x06C45D188009454F]


def test_inputs_zero_off_gasket_and_ranges():
    k = 8
    mem = fi.member_mask(k)
    ca = fi.window_values(k, fi.RULE_CA, 1)
    ht = fi.window_values(k, fi.RULE_HEAT, 1)
    assert not ca[~mem].any() and not ht[~mem].any()
    assert set(np.unique(ca).tolist()) <= {0, 1}
    assert 0.4 < ca[mem].mean() < 0.6
    assert ht.min() >= 0 and ht.max() < 1
    # window generation equals slicing the full state
    assert np.array_equal(fi.window_values(k, 1, 1, 30, 40, 50, 60), ht[40:100, 30:80])


# ------------------------------------------------------ SW and RD (Sec. 6.2)
@pytest.mark.parametrize("k", range(0, 11))
def test_gasket_mask_matches_scan(k):
    """The oracle's membership array agrees with the C oracle's cell test on
    every cell (small k) and has 3^k members (Eq. 2)."""
    mask = oracle.gasket_mask(k)
    assert int(mask.sum()) == 3 ** k
    if k <= 5:
        n = 1 << k
        for y in range(n):
            for x in range(n):
                assert mask[y, x] == oracle.member(x, y, k)


@pytest.mark.parametrize("rule,value,cell", [(0, 1, 1), (0, 0x1FF, 0xFF), (1, 0x3F800000, 1.0),
                                             (1, 0xC0490FDB, float(np.float32(-3.14159274)))])
def test_single_write_closed_form(rule, value, cell):
    """SW writes `value` on exactly the 3^k gasket cells and 0 elsewhere; its
    reduction is 3^k times the value (exact: 3^k * value needs < 53 bits)."""
    for k in range(0, 10):
        out = oracle.single_write(k, rule, value)
        nz = out != 0
        assert int(nz.sum()) == 3 ** k
        assert np.all(out[nz] == np.array(cell, dtype=out.dtype))
        tot = oracle.reduce_(k, out)
        assert tot == (3 ** k) * cell


def test_reduce_brute_force_exact():
    """RD against an exact rational sum of the members, cell by cell, on
    random uint8 and float32 states (tiny levels), with garbage off the
    gasket that must not count."""
    from fractions import Fraction
    rng = np.random.default_rng(11)
    for k in range(0, 6):
        n = 1 << k
        u8 = rng.integers(0, 256, size=(n, n), dtype=np.uint8)
        f32 = (rng.standard_normal((n, n)) * 1e3).astype(np.float32)
        want_u, want_f = 0, Fraction(0)
        for y in range(n):
            for x in range(n):
                if (x & y) == 0:
                    want_u += int(u8[y, x])
                    want_f += Fraction(float(f32[y, x]))
        assert oracle.reduce_(k, u8) == want_u
        assert oracle.reduce_(k, f32) == float(want_f)  # exactly rounded


def test_reduce_of_seeded_heat_state_is_exact():
    """Seeded heat values are multiples of 2^-24 below 1, so the sum of a
    level-10 state (59049 members) is exact in float64 and equals the
    integer sum of the 24-bit numerators times 2^-24."""
    k = 10
    st = fi.full_state(k, 1, 5)
    num = int((st.astype(np.float64) * (1 << 24)).astype(np.int64).sum())
    assert oracle.reduce_(k, st) == num / float(1 << 24)


# ------------------------------------------- compact storage (Section 7)
def _omega_of_curve(L, rb):
    """omega of the compact grid whose digits are those of L: odd mu (digit
    mu-1 of L, mu-1 even) to omega_x, even mu to omega_y (Theorem 1)."""
    wx = wy = 0
    px = py = 1
    for mu in range(1, rb + 1):
        d = L % 3
        L //= 3
        if mu % 2 == 1:
            wx += d * px
            px *= 3
        else:
            wy += d * py
            py *= 3
    return wx, wy


@pytest.mark.parametrize("k,r", [(2, 0), (4, 1), (5, 2), (6, 3), (7, 2), (8, 4), (9, 5)])
def test_compact_tile_order_is_lambda(k, r):
    """Tile L of compact storage is the block lambda(omega) of the paper's
    map (the oracle's step-by-step Theorem 1 construction, mirrored) for the
    omega whose digits are L's: its first cell sits at offset L * rho^2."""
    rb = k - r
    rho = 1 << r
    for L in range(3 ** rb):
        wx, wy = _omega_of_curve(L, rb)
        lx, ly = oracle.lambda_(rb, wx, wy)
        assert int(oracle.compact_index(k, r, lx * rho, ly * rho)) == L * rho * rho


@pytest.mark.parametrize("k,r", [(3, 0), (5, 2), (7, 3), (8, 5), (9, 7)])
def test_compact_index_bijection_and_round_trip(k, r):
    """Cells of non-empty tiles map one to one onto [0, 3^(k-r) 4^r); pack
    then unpack restores every cell of a gasket-supported state, and the
    member count is 3^k after packing (Eq. 2)."""
    n = 1 << k
    ys, xs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    live = ((xs >> r) & (ys >> r)) == 0
    idx = oracle.compact_index(k, r, xs[live], ys[live])
    size = 3 ** (k - r) * 4 ** r
    assert np.array_equal(np.sort(idx), np.arange(size))
    st = fi.full_state(k, 0, 9)
    c = oracle.pack(k, r, st)
    assert c.size == size and int(c.sum()) == int(st.sum())
    assert np.array_equal(oracle.unpack(k, r, c), st)
    ones = oracle.pack(k, r, oracle.single_write(k, 0, 1))
    assert int(ones.sum()) == 3 ** k


# --------------------------------------------------- NBB family (Sec. 3)
NBB_TABLES = {
    "gasket": ([(0, 0), (0, 1), (1, 1)], 2),
    "carpet": ([(0, 0), (1, 0), (2, 0), (0, 1), (2, 1), (0, 2), (1, 2), (2, 2)], 3),
    "vicsek": ([(1, 0), (0, 1), (1, 1), (2, 1), (1, 2)], 3),
    "xfractal": ([(0, 0), (2, 0), (1, 1), (0, 2), (2, 2)], 3),
    "cantor": ([(0, 0), (2, 0)], 3),
}


@pytest.mark.parametrize("name", sorted(NBB_TABLES))
def test_nbb_member_count_and_dimension(name):
    """Eq. 2 and Lemma 1: k^level members, Hausdorff exponent log k / log s."""
    reps, s = NBB_TABLES[name]
    k = len(reps)
    for level in range(0, 6 if s == 3 else 9):
        m = oracle.nbb_member_mask(reps, s, level)
        assert int(m.sum()) == k ** level
        if level >= 2:
            n = s ** level
            assert abs(math.log(m.sum()) / math.log(n) - math.log(k) / math.log(s)) < 1e-12


def test_nbb_carpet_golden_and_gasket_orientation():
    """The carpet at level 2 equals the hand-drawn fixture; the gasket table
    gives the paper's orientation x & (n - 1 - y) == 0 (Section 6.1)."""
    rows = [l.strip() for l in open(os.path.join(GOLDEN, "nbb_carpet_level2.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 9 and all(len(r) == 9 for r in rows)
    want = np.array([[c == "X" for c in r] for r in rows])
    reps, s = NBB_TABLES["carpet"]
    assert np.array_equal(oracle.nbb_member_mask(reps, s, 2), want)
    reps, s = NBB_TABLES["gasket"]
    for level in range(0, 8):
        n = 1 << level
        ys, xs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        assert np.array_equal(oracle.nbb_member_mask(reps, s, level), (xs & (n - 1 - ys)) == 0)


@pytest.mark.parametrize("name", sorted(NBB_TABLES))
def test_nbb_lambda_bijection_on_lemma2_grid(name):
    """Theorem 1 / Lemma 2: the map from the k^ceil(rb/2) x k^floor(rb/2)
    grid hits every non-empty block exactly once (brute force)."""
    reps, s = NBB_TABLES[name]
    k = len(reps)
    for rb in range(0, 6 if k <= 5 else 5):
        gx, gy = k ** ((rb + 1) // 2), k ** (rb // 2)
        seen = set()
        for wy in range(gy):
            for wx in range(gx):
                seen.add(oracle.nbb_lambda(reps, s, rb, wx, wy))
        blocks = oracle.nbb_member_mask(reps, s, rb)
        want = {(int(x), int(y)) for y, x in zip(*np.nonzero(blocks))}
        assert seen == want and len(want) == gx * gy


def test_nbb_lambda_gasket_matches_specialised_oracle():
    """With the gasket's table the general map is the gasket map of the C
    oracle in the paper's orientation."""
    reps, s = NBB_TABLES["gasket"]
    for rb in range(0, 9):
        gx, gy = 3 ** ((rb + 1) // 2), 3 ** (rb // 2)
        for wy in range(gy):
            for wx in range(gx):
                assert oracle.nbb_lambda(reps, s, rb, wx, wy) == oracle.lambda_paper(rb, wx, wy)


def test_nbb_ca_gasket_matches_c_oracle_mirrored():
    """On the gasket table the NBB automaton is the C oracle's automaton
    mirrored vertically (the two orientations of Section 6.1)."""
    reps, s = NBB_TABLES["gasket"]
    for k in (3, 6, 8):
        st = fi.full_state(k, 0, 21)        # (x & y) == 0 orientation
        mirrored = st[::-1, :].copy()       # x & (n-1-y) == 0 orientation
        for steps in (1, 3, 7):
            a = oracle.nbb_ca_run(reps, s, k, mirrored, steps)
            b = oracle.ca_run(k, st, steps)[::-1, :]
            assert np.array_equal(a, b), (k, steps)


@pytest.mark.parametrize("name", ["carpet", "vicsek", "xfractal"])
def test_nbb_ca_equals_textbook_life_then_mask(name):
    """On any NBB fractal the automaton equals textbook Game of Life on the
    zero-padded array (library convolution) followed by clearing the cells
    off the fractal, since cells off the fractal stay 0."""
    reps, s = NBB_TABLES[name]
    level = 4
    n = s ** level
    rng = np.random.default_rng(5)
    mask = oracle.nbb_member_mask(reps, s, level)
    st = (rng.random((n, n)) < 0.5).astype(np.uint8) * mask
    kern = np.ones((3, 3), dtype=np.int64)
    kern[1, 1] = 0
    ref = st.astype(np.int64)
    for _ in range(6):
        cnt = signal.convolve2d(ref, kern, mode="same", boundary="fill")
        ref = (((cnt == 3) | ((ref == 1) & (cnt == 2))) & mask).astype(np.int64)
    assert np.array_equal(oracle.nbb_ca_run(reps, s, level, st, 6), ref.astype(np.uint8))


def test_nbb_single_write_and_reduce():
    reps, s = NBB_TABLES["carpet"]
    for level in range(0, 5):
        sw = oracle.nbb_single_write(reps, s, level, 0x133)
        assert int((sw != 0).sum()) == 8 ** level and set(np.unique(sw)) <= {0, 0x33}
        assert oracle.nbb_reduce(reps, s, level, sw) == 0x33 * 8 ** level
        junk = sw.copy()
        junk[sw == 0] = 200
        assert oracle.nbb_reduce(reps, s, level, junk) == 0x33 * 8 ** level
