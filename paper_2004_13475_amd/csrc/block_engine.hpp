// block_engine.hpp -- the shared setup of the block engines: one wavefront
// per 64 x 64 tile, one lane per 8 x 8 block of the tile and of the part of
// its halo that can reach it within a launch.
//
// A tile of a level-k gasket is a level-3 gasket of 8 x 8 blocks (27 of
// the 64 are non-empty), and it touches the neighbouring tiles only at
// corner cells.  Within D steps a walk along the gasket from the tile gets
// only a few blocks deep into the tiles to its left, above, to its right,
// below, above right and below left, and which blocks it reaches depends
// only on which of those six tiles exist (ten patterns occur, one of them
// the lone tile of level 6).
// block_slots.inc lists the blocks per pattern, rule and D (a breadth-first
// search, gen_block_slots.py): at most 8 / 14 / 23 / 28 for heat at D = 16 /
// 24 / 32 / 36, 11 / 21 / 29 / 33 for the automaton.  Each listed block has
// a fixed lane (a constant table per rule, D and pattern), so a lane's block
// and the lanes of the blocks around it come from one table entry.  The
// steps exchange the few cells where blocks touch by ds_bpermute (two
// neighbouring blocks of a gasket touch only at corner cells); lane 63
// holds no block and stays zero, and stands for every neighbour the launch
// does not hold.  Cells near the edge of what is held see zeros for what
// lies beyond it; the damage moves one cell per step and reaches the tile
// only after more than D steps, so a launch of up to D steps leaves the
// tile exact.
#pragma once

#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

namespace blk {

constexpr int kTileLog = 6; // tiles of 64 x 64 cells
constexpr int kBlk = 8;     // blocks of 8 x 8 cells
constexpr int kTileBlk = 8; // blocks per tile side

// Halo depth in blocks for launches of up to D steps.
constexpr int halo_blocks(int D) { return (D + kBlk - 1) / kBlk; }

#include "block_slots.inc"

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Cell (i, j) of a block (column i, row j) is a member iff (i & j) == 0:
// the block's own bits and the block coordinates' bits do not overlap.
constexpr bool mem(int i, int j)
{
    return i >= 0 && j >= 0 && i < kBlk && j < kBlk && (i & j) == 0;
}

// Value v held by lane `lane` (ds_bpermute: every lane of the wavefront
// must execute it).
__device__ __forceinline__ uint32_t pull_u32(uint32_t lane, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(lane << 2), (int)v);
}

__device__ __forceinline__ float pull(uint32_t lane, float v)
{
    return __uint_as_float(pull_u32(lane, __float_as_uint(v)));
}

// Directions of the neighbouring blocks a step reads from.
enum Dir { DN = 0, DS, DW, DE, DNE, DSW, kDirs };

constexpr uint32_t kZeroLane = 63; // holds no block: every value it gives is zero

// One entry per lane: bits 0-4 and 5-9 the block's position in the region
// (the tile's first block at (H, H), H = halo_blocks(D)), bit 10 set where
// the lane holds a block, bits 16 + 8d.. the lane of the block in direction
// d (kZeroLane where the list holds none).  Lanes 0..26 hold the tile's own
// blocks in row-major order, then the pattern's halo blocks in the listed
// order.
struct SlotTable {
    uint64_t e[kMaskCount][64];
    int most; // the most lanes any pattern uses
};

template <int N>
constexpr SlotTable make_slots(const int (&halo)[kMaskCount][N][2], const int (&count)[kMaskCount],
                               int H)
{
    SlotTable s{};
    s.most = 0;
    const int dx[kDirs] = {0, 0, -1, 1, 1, -1}, dy[kDirs] = {-1, 1, 0, 0, -1, 1};
    for (int m = 0; m < kMaskCount; ++m) {
        int rx[64] = {}, ry[64] = {};
        int n = 0;
        for (int y = 0; y < kTileBlk; ++y)
            for (int x = 0; x < kTileBlk; ++x)
                if ((x & y) == 0) {
                    rx[n] = x;
                    ry[n] = y;
                    ++n;
                }
        for (int i = 0; i < count[m] && n < 64; ++i) {
            rx[n] = halo[m][i][0];
            ry[n] = halo[m][i][1];
            ++n;
        }
        s.most = n > s.most ? n : s.most;
        for (int i = 0; i < 64; ++i) {
            uint64_t e = 0;
            for (int d = 0; d < kDirs; ++d)
                e |= (uint64_t)kZeroLane << (16 + 8 * d);
            if (i < n) {
                e = (uint64_t)(rx[i] + H) | (uint64_t)(ry[i] + H) << 5 | 1ull << 10;
                for (int d = 0; d < kDirs; ++d) {
                    uint64_t l = kZeroLane;
                    for (int j = 0; j < n; ++j)
                        if (rx[j] == rx[i] + dx[d] && ry[j] == ry[i] + dy[d])
                            l = (uint64_t)j;
                    e |= l << (16 + 8 * d);
                }
            }
            s.e[m][i] = e;
        }
    }
    return s;
}

static __constant__ SlotTable kSlotsHeat16 = make_slots(kHalo_heat_16, kHaloCount_heat_16, 2);
static __constant__ SlotTable kSlotsHeat24 = make_slots(kHalo_heat_24, kHaloCount_heat_24, 3);
static __constant__ SlotTable kSlotsHeat32 = make_slots(kHalo_heat_32, kHaloCount_heat_32, 4);
static __constant__ SlotTable kSlotsHeat36 = make_slots(kHalo_heat_36, kHaloCount_heat_36, 5);
static __constant__ SlotTable kSlotsMoore16 = make_slots(kHalo_moore_16, kHaloCount_moore_16, 2);
static __constant__ SlotTable kSlotsMoore24 = make_slots(kHalo_moore_24, kHaloCount_moore_24, 3);
static __constant__ SlotTable kSlotsMoore32 = make_slots(kHalo_moore_32, kHaloCount_moore_32, 4);
static __constant__ SlotTable kSlotsMoore36 = make_slots(kHalo_moore_36, kHaloCount_moore_36, 5);
static_assert(make_slots(kHalo_heat_36, kHaloCount_heat_36, 5).most <= (int)kZeroLane &&
                  make_slots(kHalo_moore_36, kHaloCount_moore_36, 5).most <= (int)kZeroLane,
              "every table leaves the zero lane free");
static_assert(halo_blocks(36) * 2 + kTileBlk <= 32, "region positions fit five bits");
static_assert(kMaskIndex[0] >= 0 && kHaloCount_heat_36[kMaskIndex[0]] == 0 &&
                  kHaloCount_moore_36[kMaskIndex[0]] == 0,
              "a tile with no neighbours (level 6) has a pattern with no halo");

// This lane's block of the region of tile t and the lanes holding the
// blocks around it (kZeroLane where there is none, and for every direction
// of a lane that holds no block, so that it stays zero).
struct Region {
    bool active;           // this lane holds a block
    int px, py;            // its position in the region (blocks; the tile from (H, H))
    int gx, gy;            // its position in the array (blocks)
    uint32_t lane[kDirs];  // lanes of the neighbouring blocks
};

// MOORE: the automaton's eight-cell neighbourhood (otherwise the four-cell
// one of heat); D: the most steps a launch takes (16, 24, 32 or 36).  All 64
// lanes call it.
template <bool MOORE, int D>
__device__ __forceinline__ Region block_region(int k, TileXY t)
{
    static_assert(D == 16 || D == 24 || D == 32 || D == 36, "no table for these steps");
    constexpr int H = halo_blocks(D);
    const uint32_t lane = lane_id();
    // which of the neighbouring tiles exist (are inside the array and
    // non-empty); the same for the whole wavefront
    const uint32_t nt = 1u << (k - kTileLog);
    const uint32_t tx = t.x, ty = t.y;
    const bool l = tx > 0u, r = tx + 1u < nt, a = ty > 0u, b = ty + 1u < nt;
    uint32_t mask = 0u;
    mask |= (l && ((tx - 1u) & ty) == 0u) ? 1u : 0u;
    mask |= (a && (tx & (ty - 1u)) == 0u) ? 2u : 0u;
    mask |= (r && ((tx + 1u) & ty) == 0u) ? 4u : 0u;
    mask |= (b && (tx & (ty + 1u)) == 0u) ? 8u : 0u;
    mask |= (r && a && ((tx + 1u) & (ty - 1u)) == 0u) ? 16u : 0u;
    mask |= (l && b && ((tx - 1u) & (ty + 1u)) == 0u) ? 32u : 0u;
    // every mask a gasket's tile can have is listed; one that were not
    // would take the lone tile's pattern (no halo, so nothing outside the
    // array is read)
    const int m = kMaskIndex[mask] < 0 ? kMaskIndex[0] : kMaskIndex[mask];
    uint64_t e;
    if constexpr (MOORE)
        e = D == 16   ? kSlotsMoore16.e[m][lane]
            : D == 24 ? kSlotsMoore24.e[m][lane]
            : D == 32 ? kSlotsMoore32.e[m][lane]
                      : kSlotsMoore36.e[m][lane];
    else
        e = D == 16   ? kSlotsHeat16.e[m][lane]
            : D == 24 ? kSlotsHeat24.e[m][lane]
            : D == 32 ? kSlotsHeat32.e[m][lane]
                      : kSlotsHeat36.e[m][lane];
    Region g;
    g.active = ((e >> 10) & 1u) != 0u;
    g.px = (int)(e & 31u);
    g.py = (int)((e >> 5) & 31u);
    g.gx = (int)(tx << (kTileLog - 3)) - H + g.px;
    g.gy = (int)(ty << (kTileLog - 3)) - H + g.py;
#pragma unroll
    for (int d = 0; d < kDirs; ++d)
        g.lane[d] = (uint32_t)(e >> (16 + 8 * d)) & 63u;
    return g;
}

// The two-slot form on 128 x 128 tiles: 81 tile blocks and the halo of up
// to 36 steps (at most 109 blocks) over 64 lanes, two blocks per lane.
// Block q of the list (the tile's blocks row-major, then the halo) sits in
// slot q >> 6 of lane q & 63; entry q: bits 0-4 and 5-9 the block's position
// in the region (the tile from (H, H)), bit 10 set where the slot holds a
// block, bits 16 + 8d.. the list index of the block in direction d (127,
// slot 1 of lane 63, which never holds a block, where there is none).
constexpr int kTile2Log = 7;                  // tiles of 128 x 128 cells
constexpr int kTile2Blk = 1 << (kTile2Log - 3); // 16 blocks per tile side
constexpr uint32_t kZeroSlot = 127;

struct SlotTable2 {
    uint64_t e[kMaskCount][128];
    int most;
};

template <int N>
constexpr SlotTable2 make_slots2(const int (&halo)[kMaskCount][N][2], const int (&count)[kMaskCount],
                                 int H)
{
    SlotTable2 s{};
    s.most = 0;
    const int dx[kDirs] = {0, 0, -1, 1, 1, -1}, dy[kDirs] = {-1, 1, 0, 0, -1, 1};
    for (int m = 0; m < kMaskCount; ++m) {
        int rx[128] = {}, ry[128] = {};
        int n = 0;
        for (int y = 0; y < kTile2Blk; ++y)
            for (int x = 0; x < kTile2Blk; ++x)
                if ((x & y) == 0) {
                    rx[n] = x;
                    ry[n] = y;
                    ++n;
                }
        for (int i = 0; i < count[m] && n < 128; ++i) {
            rx[n] = halo[m][i][0];
            ry[n] = halo[m][i][1];
            ++n;
        }
        s.most = n > s.most ? n : s.most;
        // list index of the block at each region position (kZeroSlot: none)
        int at[32][32] = {};
        for (int y = 0; y < 32; ++y)
            for (int x = 0; x < 32; ++x)
                at[y][x] = (int)kZeroSlot;
        for (int q = 0; q < n; ++q)
            at[ry[q] + H][rx[q] + H] = q;
        for (int q = 0; q < 128; ++q) {
            uint64_t e = 0;
            for (int d = 0; d < kDirs; ++d)
                e |= (uint64_t)kZeroSlot << (16 + 8 * d);
            if (q < n) {
                e = (uint64_t)(rx[q] + H) | (uint64_t)(ry[q] + H) << 5 | 1ull << 10;
                for (int d = 0; d < kDirs; ++d) {
                    const int x = rx[q] + H + dx[d], y = ry[q] + H + dy[d];
                    const uint64_t l = (x >= 0 && y >= 0 && x < 32 && y < 32) ? (uint64_t)at[y][x]
                                                                              : kZeroSlot;
                    e |= l << (16 + 8 * d);
                }
            }
            s.e[m][q] = e;
        }
    }
    return s;
}

static __constant__ SlotTable2 kSlots2Heat36 =
    make_slots2(kHalo_heat_36_t128, kHaloCount_heat_36_t128, halo_blocks(36));
static __constant__ SlotTable2 kSlots2Moore36 =
    make_slots2(kHalo_moore_36_t128, kHaloCount_moore_36_t128, halo_blocks(36));
static_assert(make_slots2(kHalo_heat_36_t128, kHaloCount_heat_36_t128, 5).most <= (int)kZeroSlot &&
                  make_slots2(kHalo_moore_36_t128, kHaloCount_moore_36_t128, 5).most <=
                      (int)kZeroSlot,
              "the zero slot stays free");
static_assert(halo_blocks(36) * 2 + kTile2Blk <= 32, "region positions fit five bits");

// One slot of a lane in the two-slot form.
struct Slot2 {
    bool active;
    int px, py, gx, gy;
    uint32_t nb[kDirs]; // list indices of the neighbouring blocks
};

// The two slots of this lane for tile t (128 x 128) of a level-k state,
// the table of up to 36 steps (MOORE: the automaton's).  All 64 lanes call
// it.
template <bool MOORE>
__device__ __forceinline__ void block_region2(int k, TileXY t, Slot2 (&sl)[2])
{
    constexpr int H = halo_blocks(36);
    const uint32_t lane = lane_id();
    const uint32_t nt = 1u << (k - kTile2Log);
    const uint32_t tx = t.x, ty = t.y;
    const bool l = tx > 0u, r = tx + 1u < nt, a = ty > 0u, b = ty + 1u < nt;
    uint32_t mask = 0u;
    mask |= (l && ((tx - 1u) & ty) == 0u) ? 1u : 0u;
    mask |= (a && (tx & (ty - 1u)) == 0u) ? 2u : 0u;
    mask |= (r && ((tx + 1u) & ty) == 0u) ? 4u : 0u;
    mask |= (b && (tx & (ty + 1u)) == 0u) ? 8u : 0u;
    mask |= (r && a && ((tx + 1u) & (ty - 1u)) == 0u) ? 16u : 0u;
    mask |= (l && b && ((tx - 1u) & (ty + 1u)) == 0u) ? 32u : 0u;
    const int m = kMaskIndex[mask] < 0 ? kMaskIndex[0] : kMaskIndex[mask];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const uint64_t e = MOORE ? kSlots2Moore36.e[m][s * 64 + lane] : kSlots2Heat36.e[m][s * 64 + lane];
        sl[s].active = ((e >> 10) & 1u) != 0u;
        sl[s].px = (int)(e & 31u);
        sl[s].py = (int)((e >> 5) & 31u);
        sl[s].gx = (int)(tx << (kTile2Log - 3)) - H + sl[s].px;
        sl[s].gy = (int)(ty << (kTile2Log - 3)) - H + sl[s].py;
#pragma unroll
        for (int d = 0; d < kDirs; ++d)
            sl[s].nb[d] = (uint32_t)(e >> (16 + 8 * d)) & 127u;
    }
}

// Where a state's cells live.  ArrayLayout: the n x n array, row-major.
struct ArrayLayout {
    int64_t row_bytes; // bytes per array row
    int S;             // bytes per cell
    TileXY t;          // the tile the wavefront advances
    int tile_log = kTileLog; // its side, log2
    __device__ __forceinline__ int64_t block_off(int gx, int gy) const
    {
        return (int64_t)(gy * kBlk) * row_bytes + (int64_t)gx * kBlk * S;
    }
    __device__ __forceinline__ int64_t pitch() const { return row_bytes; }
    __device__ __forceinline__ int64_t tile_row(int r) const
    {
        return (((int64_t)t.y << tile_log) + r) * row_bytes + ((int64_t)t.x << tile_log) * S;
    }
};

// The base-3 reading of a byte's bits: sum of 3^i over its set bits i.
struct Base3Bytes {
    uint32_t v[256];
};
constexpr Base3Bytes make_base3_bytes()
{
    Base3Bytes b{};
    for (int x = 0; x < 256; ++x) {
        uint32_t s = 0, p = 1;
        for (int i = 0; i < 8; ++i, p *= 3)
            s += ((x >> i) & 1) ? p : 0u;
        b.v[x] = s;
    }
    return b;
}
static __constant__ Base3Bytes kBase3Bytes = make_base3_bytes();

// lambda^-1 of tile (x, y) of a level-rb tile space (rb <= 16): its curve
// index, whose base-3 digit mu is 2 where bit mu of x is set, 0 where that
// of y is, 1 elsewhere, i.e. (3^rb - 1) / 2 + B(x) - B(y) with B the base-3
// reading of a bit pattern.  Wave-uniform arguments keep it in scalar
// registers.  Coordinates outside the space give some index (unused).
__device__ __forceinline__ uint32_t curve_index(uint32_t x, uint32_t y, int rb)
{
    auto b3 = [](uint32_t v) {
        return kBase3Bytes.v[v & 255u] + 6561u * kBase3Bytes.v[(v >> 8) & 255u];
    };
    return (pow3_u32((uint32_t)rb) - 1u) / 2u + b3(x) - b3(y);
}

// Compact storage: the non-empty 64 x 64 tiles in curve order, each
// row-major; a launch reads blocks of the tile and of its left, above,
// right, below, above-right and below-left neighbours, found by their curve
// indices.
struct CompactLayout {
    int S; // bytes per cell
    TileXY t;
    uint32_t own, left, above, right, below, aright, bleft;
    __device__ __forceinline__ int64_t block_off(int gx, int gy) const
    {
        const int dx = (gx >> 3) - (int)t.x, dy = (gy >> 3) - (int)t.y;
        uint32_t i = own;
        i = dx < 0 ? (dy > 0 ? bleft : left) : i;
        i = dx > 0 ? (dy < 0 ? aright : right) : i;
        i = dx == 0 ? (dy < 0 ? above : (dy > 0 ? below : own)) : i;
        return ((((int64_t)i << (2 * kTileLog)) + ((int64_t)((gy & 7) * kBlk) << kTileLog) +
                 (gx & 7) * kBlk) *
                S);
    }
    __device__ __forceinline__ int64_t pitch() const { return (int64_t)S << kTileLog; }
    __device__ __forceinline__ int64_t tile_row(int r) const
    {
        return (((int64_t)own << (2 * kTileLog)) + ((int64_t)r << kTileLog)) * S;
    }
};

// The compact layout of tile t, curve index L, of a level-rb tile space.
__device__ __forceinline__ CompactLayout compact_layout(TileXY t, uint32_t L, int rb, int S)
{
    CompactLayout c;
    c.S = S;
    c.t = t;
    c.own = L;
    c.left = curve_index(t.x - 1u, t.y, rb);
    c.above = curve_index(t.x, t.y - 1u, rb);
    c.right = curve_index(t.x + 1u, t.y, rb);
    c.below = curve_index(t.x, t.y + 1u, rb);
    c.aright = curve_index(t.x + 1u, t.y - 1u, rb);
    c.bleft = curve_index(t.x - 1u, t.y + 1u, rb);
    return c;
}

} // namespace blk

} // namespace fractal

