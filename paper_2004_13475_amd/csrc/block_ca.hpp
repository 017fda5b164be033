// block_ca.hpp -- the block engine of the uint8 B3/S23 automaton (one
// wavefront per 64 x 64 tile, one lane per non-empty 8 x 8 block; the
// shared setup is in block_engine.hpp).  A lane keeps its block as a 64-bit
// board (bit 8j + i holds cell (i, j)) and advances it with bitwise
// operations: the eight neighbour boards are the board shifted, with the
// cells of the neighbouring blocks that touch it shifted in, and a
// bit-sliced adder counts them.  In a gasket only these cells of other
// blocks touch a block's members: the cell (0,7) of the block above and of
// the block above right, (7,0) of the block to the left and of the block
// below left, (0,0) and (0,1) of the block to the right, (0,0) and (1,0) of
// the block below; a step reads the words that hold them from six lanes.
// The finished tile is assembled in LDS (4 KB per wavefront) and written a
// whole 64-byte row per lane.
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
constexpr uint64_t kCol0 = 0x0101010101010101ull;
constexpr uint64_t kCol7 = 0x8080808080808080ull;

// The low bits of bytes 0..3 of v gathered into bits 0..3 (the products of
// the four terms land on distinct bits, so nothing carries into 28..31).
__device__ __forceinline__ uint32_t pack4(uint32_t v) { return (v * 0x10204080u) >> 28; }
// Bits 0..3 of x spread to the low bits of bytes 0..3 (same argument).
__device__ __forceinline__ uint32_t unpack4(uint32_t x)
{
    return ((x & 0xFu) * 0x00204081u) & 0x01010101u;
}

// Three-input xor and majority of 64-bit boards, one v_bitop3 per 32-bit
// half (both functions are symmetric in their inputs).
__device__ __forceinline__ uint64_t xor3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32),
                                                    (uint32_t)(c >> 32), 0x96);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t maj3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0xE8);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32),
                                                    (uint32_t)(c >> 32), 0xE8);
    return ((uint64_t)hi << 32) | lo;
}

// One B3/S23 step of board b.  nrow: row 7 of the block above (bits 0..7);
// srow: row 0 of the block below (bits 0..7); wcol: column 7 of the block to
// the left in column 0 (rows 0..3); ecol: column 0 of the block to the right
// in column 7 (rows 0..3); ne: cell (0,7) of the block above right; sw: cell
// (7,0) of the block below left.  Cells outside these are not members or
// touch no member of this block.
__device__ __forceinline__ uint64_t life_step(uint64_t b, uint64_t nrow, uint64_t srow,
                                              uint64_t wcol, uint64_t ecol, uint64_t ne,
                                              uint64_t sw)
{
    const uint64_t nb = (b << 8) | nrow;         // cell (i, j-1)
    const uint64_t sb = (b >> 8) | (srow << 56); // cell (i, j+1)
    const uint64_t n1 = nb;
    const uint64_t n2 = sb;
    const uint64_t n3 = ((b << 1) & ~kCol0) | wcol;                       // (i-1, j)
    const uint64_t n4 = ((b >> 1) & ~kCol7) | ecol;                       // (i+1, j)
    const uint64_t n5 = ((nb << 1) & ~kCol0) | (wcol << 8);               // (i-1, j-1)
    const uint64_t n6 = ((nb >> 1) & ~kCol7) | (ecol << 8) | (ne << 7);   // (i+1, j-1)
    const uint64_t n7 = ((sb << 1) & ~kCol0) | (wcol >> 8) | (sw << 56);  // (i-1, j+1)
    const uint64_t n8 = ((sb >> 1) & ~kCol7) | (ecol >> 8);               // (i+1, j+1)
    // bit-sliced sum of the eight boards (full adders: sum = xor3, carry =
    // majority): count = s0 + 2 s1 + 4 (f0 + f1)
    const uint64_t a1 = xor3(n1, n2, n3), c1 = maj3(n1, n2, n3);
    const uint64_t a2 = xor3(n4, n5, n6), c2 = maj3(n4, n5, n6);
    const uint64_t a3 = n7 ^ n8, c3 = n7 & n8;
    const uint64_t s0 = xor3(a1, a2, a3), c4 = maj3(a1, a2, a3);
    const uint64_t t = xor3(c1, c2, c3), f0 = maj3(c1, c2, c3);
    const uint64_t s1 = t ^ c4, f1 = t & c4;
    // B3/S23: alive next iff count == 3, or count == 2 and alive now
    return kMembers & s1 & ~(f0 | f1) & (s0 | b);
}

} // namespace blk

// One wavefront advances the tile t of a level-k automaton state `steps`
// steps (1..16), src -> dst; all 64 lanes call it.
template <int FL>
__device__ __forceinline__ void block_ca_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                              TileXY t, int steps)
{
    using namespace blk;
    const Region g = block_region(k, t);
    const int n = 1 << k;
    const int64_t base = (int64_t)(g.gy * kBlk) * n + (int64_t)g.gx * kBlk;
    // load: 8 bytes a row (rows 4..7 hold members in their first four)
    uint64_t b = 0;
    {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        using gu2 = const __attribute__((address_space(1))) u32x2;
        const uint8_t *src = src_state + (g.active ? base : 0);
        static_for<0, kBlk>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const u32x2 v = *(gu2 *)(src + (int64_t)j * n);
            const uint64_t row = pack4(v[0]) | (pack4(v[1]) << 4);
            b |= row << (8 * j);
        });
        b = g.active ? (b & kMembers) : 0ull;
    }
    auto step = [&](uint64_t cur) -> uint64_t {
        const uint32_t lo = (uint32_t)cur, hi = (uint32_t)(cur >> 32);
        // every lane takes part in every exchange (a lane with no such
        // neighbour reads itself and drops the value)
        uint32_t vn = pull_u32(g.lane[DN], hi), vs = pull_u32(g.lane[DS], lo);
        uint32_t vw = pull_u32(g.lane[DW], lo), ve = pull_u32(g.lane[DE], lo);
        uint32_t vne = pull_u32(g.lane[DNE], hi), vsw = pull_u32(g.lane[DSW], lo);
        vn = g.ok[DN] ? vn : 0u;
        vs = g.ok[DS] ? vs : 0u;
        vw = g.ok[DW] ? vw : 0u;
        ve = g.ok[DE] ? ve : 0u;
        vne = g.ok[DNE] ? vne : 0u;
        vsw = g.ok[DSW] ? vsw : 0u;
        return life_step(cur, (vn >> 24) & 0xFFu, vs & 0xFFu, (vw >> 7) & 0x01010101u,
                         (uint64_t)(ve & 0x01010101u) << 7, (vne >> 24) & 1u, (vsw >> 7) & 1u);
    };
    for (int s = 0; s < steps; ++s)
        b = step(b);

    // Store: a 64-byte segment is a whole tile row (eight blocks), so the
    // wavefront assembles its tile in LDS (zeros where blocks are empty)
    // and each lane writes one tile row with four 16-byte stores.
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
    const bool inner = g.active && g.px >= kHaloBlk && g.px < kHaloBlk + kTileBlk &&
                       g.py >= kHaloBlk && g.py < kHaloBlk + kTileBlk;
    if (inner) {
        const int w0 = ((g.py - kHaloBlk) * kBlk) * 16 + (g.px - kHaloBlk) * 2;
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
        // lane r: tile row r (every row of a non-empty tile holds members)
        const int64_t y = ((int64_t)t.y << kTileLog) + lane;
        u32x4v *p = reinterpret_cast<u32x4v *>(dst_state + y * n + ((int64_t)t.x << kTileLog));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4v v = *reinterpret_cast<const u32x4v *>(my + lane * 16 + 4 * q);
            if constexpr (FL & TILE_NT_STORE)
                __builtin_nontemporal_store(v, p + q);
            else
                p[q] = v;
        }
    }
}

} // namespace fractal
