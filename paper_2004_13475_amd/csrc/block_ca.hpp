// block_ca.hpp -- the block engine of the uint8 B3/S23 automaton (one
// wavefront per 64 x 64 tile, one lane per 8 x 8 block; the shared setup is
// in block_engine.hpp).  A lane loads and stores its block as a 64-bit
// board (bit 8j + i holds cell (i, j)) and steps it as two words, one of
// the even rows and one of the odd rows (byte m of each: row 2m, row
// 2m + 1), so that the rows above and below a row of one word are the other
// word, shifted by a row for one of the two directions only.  A step first
// sums each cell's row neighbours, (i-1, j) + (i+1, j), and the same with
// the cell itself; the rows above and below contribute their three-cell
// sums, taken from this board or, for row 0 and row 7, from the lanes of
// the blocks above and below, whose sums already hold the diagonal blocks'
// cells.  In a gasket only these cells of other blocks touch a block's
// members: (7,0) of the block to the left, column 0 of the block to the
// right, (0,7) of the blocks above and above right, and row 0 of the block
// below with (7,0) of the block below left.  Each lane publishes what its
// neighbours read in three words (column 0; row 7's sums with cell (0,7);
// row 0's sums with row 0), so a step costs four lane exchanges.  The finished tile is assembled in LDS (4 KB
// per wavefront) and written four lanes to a 64-byte row.
#pragma once

#include "block_engine.hpp"

namespace fractal {

namespace blk {

// The members of a block as a board.
constexpr uint64_t member_board()
{
    uint64_t m = 0;
    for (int j = 0; j < kBlk; ++j)
        for (int i = 0; i < kBlk; ++i)
            if ((i & j) == 0)
                m |= 1ull << (8 * j + i);
    return m;
}
constexpr uint64_t kMembers = member_board();

// The low bits of bytes 0..3 of v gathered into bits 0..3 (the products of
// the four terms land on distinct bits, so nothing carries into 28..31).
__device__ __forceinline__ uint32_t pack4(uint32_t v) { return (v * 0x10204080u) >> 28; }
// Bits 0..3 of x spread to the low bits of bytes 0..3 (same argument).
__device__ __forceinline__ uint32_t unpack4(uint32_t x)
{
    return ((x & 0xFu) * 0x00204081u) & 0x01010101u;
}

// Bytes 0, 2, 4, 6 (even) or 1, 3, 5, 7 (odd) of a board as one word.
constexpr uint32_t rows_of(uint64_t b, int odd)
{
    uint32_t w = 0;
    for (int m = 0; m < 4; ++m)
        w |= (uint32_t)((b >> (8 * (2 * m + odd))) & 0xFFu) << (8 * m);
    return w;
}
constexpr uint32_t kMembersLo = rows_of(kMembers, 0), kMembersHi = rows_of(kMembers, 1);

// Three-input xor and majority (one v_bitop3 each; both are symmetric in
// their inputs).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
// The bits of a where m is set, of b elsewhere (one v_bitop3, which also
// keeps the compiler from splitting the two halves apart for its users).
__device__ __forceinline__ uint32_t merge(uint32_t m, uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_bitop3_b32(m, a, b, 0xCA);
}
// The low word of (hi:lo) >> s.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

struct Board {
    uint32_t lo, hi; // rows 0, 2, 4, 6 and rows 1, 3, 5, 7, a byte each
};
// A 64-bit board as even and odd rows, and back (one v_perm each).
__device__ __forceinline__ Board split_rows(uint64_t b)
{
    const uint32_t l = (uint32_t)b, h = (uint32_t)(b >> 32);
    return Board{__builtin_amdgcn_perm(h, l, 0x06040200u), __builtin_amdgcn_perm(h, l, 0x07050301u)};
}
__device__ __forceinline__ uint64_t join_rows(Board b)
{
    const uint32_t l = __builtin_amdgcn_perm(b.hi, b.lo, 0x05010400u);
    const uint32_t h = __builtin_amdgcn_perm(b.hi, b.lo, 0x07030602u);
    return ((uint64_t)h << 32) | l;
}

// A board's row sums: per cell, two-bit sums of (i-1, j) + (i, j) + (i+1, j)
// (x0, x1) and of (i-1, j) + (i+1, j) (c0, c1), even and odd rows.
struct RowSums {
    uint32_t x0lo, x1lo, x0hi, x1hi, c0lo, c1lo, c0hi, c1hi;
};

// Column 0 of a board as the block to its left reads it: the even rows'
// cells at bits 8m, the odd rows' at bits 8m + 1.
__device__ __forceinline__ uint32_t column0(Board b)
{
    return merge(0x01010101u, b.lo, b.hi << 1);
}

// w: the even rows of the block to the left; e: column0() of the block to
// the right.  The cells (i-1, j) and (i+1, j) are the board shifted along
// its rows, with column 7 of the block to the left (a member in row 0 only)
// and column 0 of the block to the right shifted in; the odd rows hold no
// member in column 7, so their left shift spills nothing.
__device__ __forceinline__ RowSums row_sums(Board b, uint32_t w, uint32_t e)
{
    const uint32_t llo = merge(0xFEFEFEFEu, b.lo << 1, w >> 7), lhi = b.hi << 1;
    const uint32_t rlo = merge(0x7F7F7F7Fu, b.lo >> 1, e << 7);
    const uint32_t rhi = merge(0x7F7F7F7Fu, b.hi >> 1, e << 6);
    RowSums r;
    r.x0lo = xor3(llo, b.lo, rlo);
    r.x1lo = maj3(llo, b.lo, rlo);
    r.x0hi = xor3(lhi, b.hi, rhi);
    r.x1hi = maj3(lhi, b.hi, rhi);
    r.c0lo = llo ^ rlo;
    r.c1lo = llo & rlo;
    r.c0hi = lhi ^ rhi;
    r.c1hi = lhi & rhi;
    return r;
}

// The step from the row sums and the rows above and below: n0, n1 the
// sums of row 7 of the block above (in their top bytes), s0, s1 those of
// row 0 of the block below (in their low bytes), with the corner cells of
// the diagonal blocks already in.  Above an even row lies the odd row of
// the byte before (row 7 of the block above for row 0), below it the odd
// row of the same byte; above an odd row the even row of the same byte,
// below it the even row of the next byte (row 0 of the block below for
// row 7).  Neighbours = u + d + c (at most 3 + 3 +
// 2): bit 0 is the xor t of the low planes; with their carry k and the
// high planes' sum p and carry q, the count is 2 or 3 iff k + p + 2q == 1,
// i.e. (k ^ p) & ~q.  Alive next iff the count is 3, or 2 and alive now;
// non-members stay zero.
__device__ __forceinline__ Board life_finish(Board b, const RowSums &r, uint32_t n0, uint32_t n1,
                                             uint32_t s0, uint32_t s1)
{
    const uint32_t u0lo = funnel(r.x0hi, n0, 24), u0hi = r.x0lo;
    const uint32_t u1lo = funnel(r.x1hi, n1, 24), u1hi = r.x1lo;
    const uint32_t d0lo = r.x0hi, d0hi = funnel(s0, r.x0lo, 8);
    const uint32_t d1lo = r.x1hi, d1hi = funnel(s1, r.x1lo, 8);
    auto rule = [](uint32_t u0, uint32_t d0, uint32_t c0, uint32_t u1, uint32_t d1, uint32_t c1,
                   uint32_t self, uint32_t members) {
        const uint32_t t = xor3(u0, d0, c0), k = maj3(u0, d0, c0);
        const uint32_t p = xor3(u1, d1, c1), q = maj3(u1, d1, c1);
        return (k ^ p) & ~q & ((t | self) & members);
    };
    Board nx;
    nx.lo = rule(u0lo, d0lo, r.c0lo, u1lo, d1lo, r.c1lo, b.lo, kMembersLo);
    nx.hi = rule(u0hi, d0hi, r.c0hi, u1hi, d1hi, r.c1hi, b.hi, kMembersHi);
    return nx;
}

// What the block below reads: bytes [0, row 7, x0 of row 7, x1 of row 7]
// (the raw row holds one member, cell (0,7), at bit 8).  What the block
// above reads: [x1 of row 0, x0 of row 0, row 0, 0] (cell (7,0) at bit 23).
// One v_perm gathers two sources' bytes (selector 12 gives a zero byte).
__device__ __forceinline__ uint32_t down_word(Board b, const RowSums &r)
{
    return __builtin_amdgcn_perm(b.hi, __builtin_amdgcn_perm(r.x1hi, r.x0hi, 0x07030C0Cu), 0x0302070Cu);
}
__device__ __forceinline__ uint32_t up_word(Board b, const RowSums &r)
{
    return __builtin_amdgcn_perm(b.lo, __builtin_amdgcn_perm(r.x0lo, r.x1lo, 0x0C0C0400u), 0x0C040100u);
}

// Where a lane reads each step and how it unpacks it.  The row above comes
// from the block above when that block is held (its row 7 sums already
// hold the corner cell of the block above right), else from the block
// above right (its cell (0,7) alone, row sums zero); the same below.
struct Links {
    uint32_t w, e, n, s; // lanes (or list entries) read
    uint32_t shn, mn;    // n0 = word << shn, n1 = word & mn
    uint32_t shs, ms;    // s0 = word >> shs, s1 = word & ms
};
__device__ __forceinline__ Links make_links(uint32_t w, uint32_t e, uint32_t n, uint32_t ne, bool have_n,
                                            uint32_t s, uint32_t sw, bool have_s)
{
    Links k;
    k.w = w;
    k.e = e;
    k.n = have_n ? n : ne;
    k.shn = have_n ? 8u : 23u;
    k.mn = have_n ? ~0u : 0u;
    k.s = have_s ? s : sw;
    k.shs = have_s ? 8u : 23u;
    k.ms = have_s ? ~0u : 0u;
    return k;
}
// n0, n1, s0, s1 for life_finish from the words read from above and below
__device__ __forceinline__ Board life_from(Board b, const RowSums &r, uint32_t vn, uint32_t vs,
                                           const Links &k)
{
    return life_finish(b, r, vn << k.shn, vn & k.mn, vs >> k.shs, vs & k.ms);
}

// One B3/S23 step of board b, four lane exchanges.  Every lane of the
// wavefront calls it.
__device__ __forceinline__ Board life_step(Board b, const Links &k)
{
    const uint32_t w = pull_u32(k.w, b.lo), e = pull_u32(k.e, column0(b));
    const RowSums r = row_sums(b, w, e);
    const uint32_t vn = pull_u32(k.n, down_word(b, r)), vs = pull_u32(k.s, up_word(b, r));
    return life_from(b, r, vn, vs, k);
}

// The board of the block whose first cell is at src (rows P bytes apart;
// rows 4..7 hold members in their first four cells); zero where the lane
// holds no block.
__device__ __forceinline__ uint64_t load_board(const uint8_t *src, int64_t P, bool active)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    using gu2 = const __attribute__((address_space(1))) u32x2;
    uint64_t b = 0;
    static_for<0, kBlk>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const u32x2 v = *(gu2 *)(src + j * P);
        const uint64_t row = pack4(v[0]) | (pack4(v[1]) << 4);
        b |= row << (8 * j);
    });
    return active ? (b & kMembers) : 0ull;
}

} // namespace blk

// One wavefront advances the tile t of a level-k automaton state `steps`
// steps (1..D), src -> dst, the cells where `lay` puts them; all 64 lanes
// call it.
template <int FL, int D, class Layout>
__device__ __forceinline__ void block_ca_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                              TileXY t, int steps, const Layout &lay)
{
    using namespace blk;
    constexpr int H = halo_blocks(D);
    const Region g = block_region<true, D>(k, t);
    const int64_t base = lay.block_off(g.gx, g.gy);
    const int64_t P = lay.pitch(); // bytes between a block's rows
    // load: 8 bytes a row (rows 4..7 hold members in their first four)
    uint64_t b = load_board(src_state + (g.active ? base : 0), P, g.active);
    // the diagonal lanes only where the block relaying their corner cell is
    // not held
    const uint32_t have_n = pull_u32(g.lane[DN], g.active ? 1u : 0u);
    const uint32_t have_s = pull_u32(g.lane[DS], g.active ? 1u : 0u);
    const Links links = make_links(g.lane[DW], g.lane[DE], g.lane[DN], g.lane[DNE], have_n != 0u,
                                   g.lane[DS], g.lane[DSW], have_s != 0u);
    Board cur = split_rows(b);
    for (int s = 0; s < steps; ++s)
        cur = life_step(cur, links);
    b = join_rows(cur);

    // Store: a 64-byte segment is a whole tile row (eight blocks), so the
    // wavefront assembles its tile in LDS (zeros where blocks are empty)
    // and writes it in 16-byte pieces, whole rows per instruction.
    __shared__ uint32_t rows[4][64 * 16]; // per wavefront: 64 rows of 64 bytes
    uint32_t *my = rows[threadIdx.x >> 6];
    const uint32_t lane = lane_id();
    typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < 4; ++q)
        *reinterpret_cast<u32x4v *>(my + lane * 16 + 4 * q) = u32x4v{0u, 0u, 0u, 0u};
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool inner = g.active && g.px >= H && g.px < H + kTileBlk && g.py >= H &&
                       g.py < H + kTileBlk;
    if (inner) {
        const int w0 = ((g.py - H) * kBlk) * 16 + (g.px - H) * 2;
        static_for<0, kBlk>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const uint32_t row = (uint32_t)(b >> (8 * j)) & 0xFFu;
            my[w0 + j * 16] = unpack4(row);
            my[w0 + j * 16 + 1] = unpack4(row >> 4);
        });
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
        // four lanes per tile row, so that each store instruction writes 16
        // whole 64-byte rows (every row of a non-empty tile holds members)
        const uint32_t quarter = lane & 3u, r0 = lane >> 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t r = 16u * q + r0;
            u32x4v *p = reinterpret_cast<u32x4v *>(dst_state + lay.tile_row((int)r)) + quarter;
            const u32x4v v = *reinterpret_cast<const u32x4v *>(my + r * 16 + 4 * quarter);
            if constexpr (FL & TILE_NT_STORE)
                __builtin_nontemporal_store(v, p);
            else
                *p = v;
        }
    }
}

// One wavefront advances the 128 x 128 tile t of a level-k automaton state
// `steps` steps (1..36), src -> dst, two blocks per lane; all 64 lanes call
// it.  Each value a step reads from a neighbouring block is read from both
// slots of the lane that holds it, keeping the one of the block's slot.
template <int FL, class Layout>
__device__ __forceinline__ void block2_ca_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                               TileXY t, int steps, const Layout &lay)
{
    using namespace blk;
    constexpr int H = halo_blocks(36);
    Slot2 sl[2];
    block_region2<true>(k, t, sl);
    const int64_t P = lay.pitch();
    Board cur[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const uint64_t b = load_board(
            src_state + (sl[s].active ? lay.block_off(sl[s].gx, sl[s].gy) : 0), P, sl[s].active);
        cur[s] = split_rows(b);
    }
    // the value of `v` (per slot) held by list entry q
    auto pull2 = [](uint32_t q, uint32_t v0, uint32_t v1) {
        const uint32_t x0 = pull_u32(q & 63u, v0), x1 = pull_u32(q & 63u, v1);
        return (q & 64u) ? x1 : x0;
    };
    // the diagonal blocks only where the block relaying their corner cell
    // is not held
    Links links[2];
    const uint32_t a0 = sl[0].active ? 1u : 0u, a1 = sl[1].active ? 1u : 0u;
#pragma unroll
    for (int s = 0; s < 2; ++s)
        links[s] = make_links(sl[s].nb[DW], sl[s].nb[DE], sl[s].nb[DN], sl[s].nb[DNE],
                              pull2(sl[s].nb[DN], a0, a1) != 0u, sl[s].nb[DS], sl[s].nb[DSW],
                              pull2(sl[s].nb[DS], a0, a1) != 0u);
    for (int st = 0; st < steps; ++st) {
        RowSums r[2];
        const uint32_t c0 = column0(cur[0]), c1 = column0(cur[1]);
#pragma unroll
        for (int s = 0; s < 2; ++s)
            r[s] = row_sums(cur[s], pull2(links[s].w, cur[0].lo, cur[1].lo), pull2(links[s].e, c0, c1));
        const uint32_t dn0 = down_word(cur[0], r[0]), dn1 = down_word(cur[1], r[1]);
        const uint32_t up0 = up_word(cur[0], r[0]), up1 = up_word(cur[1], r[1]);
        Board nx[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
            nx[s] = life_from(cur[s], r[s], pull2(links[s].n, dn0, dn1), pull2(links[s].s, up0, up1),
                              links[s]);
        cur[0] = nx[0];
        cur[1] = nx[1];
    }

    // Store: a tile row is 128 bytes (sixteen blocks); the wavefront
    // assembles the tile in LDS a quarter (32 rows, 4 KB) at a time, zeros
    // where blocks are empty, and writes each quarter eight lanes to a row
    // (4 KB of LDS per wavefront keeps eight wavefronts on a SIMD).
    constexpr int kRows = 32, kBlkRows = kRows / kBlk;
    __shared__ uint32_t part[4][kRows * 32]; // per wavefront: 32 rows of 128 bytes
    uint32_t *my = part[threadIdx.x >> 6];
    const uint32_t lane = lane_id();
    typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
    auto wave_sync = []() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const uint64_t fin[2] = {join_rows(cur[0]), join_rows(cur[1])};
#pragma unroll
    for (int h = 0; h < kTile2Blk / kBlkRows; ++h) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<u32x4v *>(my + lane * 16 + 4 * q) = u32x4v{0u, 0u, 0u, 0u};
        wave_sync();
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int bx = sl[s].px - H, by = sl[s].py - H - kBlkRows * h;
            if (sl[s].active && bx >= 0 && bx < kTile2Blk && by >= 0 && by < kBlkRows) {
                const int w0 = by * kBlk * 32 + bx * 2;
                static_for<0, kBlk>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    const uint32_t row = (uint32_t)(fin[s] >> (8 * j)) & 0xFFu;
                    my[w0 + j * 32] = unpack4(row);
                    my[w0 + j * 32 + 1] = unpack4(row >> 4);
                });
            }
        }
        wave_sync();
        // eight lanes per 128-byte row: each store instruction writes eight
        // whole rows; rows 64..127 hold no member in columns 64..127 (that
        // quarter of a tile is empty, as the 64 x 64 tile there is), so only
        // their first 64 bytes are written
        const uint32_t chunk = lane & 7u, r0 = lane >> 3;
        if (kRows * h < 64 || chunk < 4u) {
#pragma unroll
            for (int q = 0; q < kRows / 8; ++q) {
                const uint32_t r = 8u * q + r0;
                u32x4v *p =
                    reinterpret_cast<u32x4v *>(dst_state + lay.tile_row((int)(kRows * h + r))) + chunk;
                const u32x4v v = *reinterpret_cast<const u32x4v *>(my + r * 32 + 4 * chunk);
                if constexpr (FL & TILE_NT_STORE)
                    __builtin_nontemporal_store(v, p);
                else
                    *p = v;
            }
        }
        wave_sync();
    }
}

// The n x n array form.
template <int FL, int D>
__device__ __forceinline__ void block_ca_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                              TileXY t, int steps)
{
    block_ca_tile<FL, D>(src_state, dst_state, k, t, steps, blk::ArrayLayout{(int64_t)1 << k, 1, t});
}

} // namespace fractal
