// block_engine.hpp -- the shared setup of the block engines: one wavefront
// per 64 x 64 tile, one lane per non-empty 8 x 8 block of the tile and its
// halo of two blocks (16 cells) on each side.
//
// A tile of a level-k gasket is a level-3 gasket of 8 x 8 blocks, and its
// halo holds more non-empty blocks of the neighbouring tiles: at most 54 in
// the 12 x 12 blocks of the region, so one block per lane fits one
// wavefront.  Lanes take the region's non-empty blocks in row-major order,
// each lane learns which lanes hold the blocks around its own, and the
// steps exchange the few cells where blocks touch by ds_bpermute (in a
// gasket two neighbouring blocks touch only at corner cells).  Blocks near
// the region's edge see zeros for what lies outside it; the damage moves
// one cell per step and the tile is 16 cells in, so a launch of up to 16
// steps leaves the tile exact.
#pragma once

#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

namespace blk {

constexpr int kTileLog = 6;   // tiles of 64 x 64 cells
constexpr int kBlk = 8;       // blocks of 8 x 8 cells
constexpr int kTileBlk = 8;   // blocks per tile side
constexpr int kHaloBlk = 2;   // halo blocks per side (16 cells: up to 16 steps)
constexpr int kReg = kTileBlk + 2 * kHaloBlk; // region side in blocks
constexpr int kPos = kReg * kReg;             // 144 block positions

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Cell (i, j) of a block (column i, row j) is a member iff (i & j) == 0:
// the block's own bits and the block coordinates' bits do not overlap.
constexpr bool mem(int i, int j)
{
    return i >= 0 && j >= 0 && i < kBlk && j < kBlk && (i & j) == 0;
}

// Index of the r-th set bit (0-based) of v.
__device__ __forceinline__ uint32_t select_bit(uint64_t v, uint32_t r)
{
    uint32_t pos = 0u;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const uint64_t low = v & ((1ull << s) - 1ull);
        const uint32_t c = (uint32_t)__builtin_popcountll(low);
        if (r >= c) {
            r -= c;
            v >>= s;
            pos += (uint32_t)s;
        }
    }
    return pos;
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

// This lane's block of the region of tile t and the lanes holding the
// blocks around it (this lane itself where there is no such block: outside
// the region or empty).
struct Region {
    bool active;           // this lane holds a block
    int px, py;            // its position in the region (blocks)
    int gx, gy;            // its position in the array (blocks)
    uint32_t lane[kDirs];  // lanes of the neighbouring blocks
    bool ok[kDirs];        // whether each exists
};

// All 64 lanes call it.
__device__ __forceinline__ Region block_region(int k, TileXY t)
{
    const uint32_t lane = lane_id();
    // the region's non-empty blocks, in row-major order of the 12 x 12
    // positions (three ballots of 64 positions)
    const int nbl = 1 << (k - 3); // blocks per array side
    const int bx0 = (int)(t.x << (kTileLog - 3)) - kHaloBlk;
    const int by0 = (int)(t.y << (kTileLog - 3)) - kHaloBlk;
    // (three scalars, not an array: a selected array element would be
    // read from private memory)
    auto nonempty = [&](int p) {
        const int gx = bx0 + p % kReg, gy = by0 + p / kReg;
        return p < kPos && gx >= 0 && gy >= 0 && gx < nbl && gy < nbl && (gx & gy) == 0;
    };
    const uint64_t m0 = __builtin_amdgcn_ballot_w64(nonempty((int)lane));
    const uint64_t m1 = __builtin_amdgcn_ballot_w64(nonempty((int)lane + 64));
    const uint64_t m2 = __builtin_amdgcn_ballot_w64(nonempty((int)lane + 128));
    const uint32_t c0 = (uint32_t)__builtin_popcountll(m0);
    const uint32_t c1n = (uint32_t)__builtin_popcountll(m1);
    const uint32_t nblocks = c0 + c1n + (uint32_t)__builtin_popcountll(m2);
    const bool active = lane < nblocks;
    // this lane's block: the lane-th non-empty position
    uint32_t pos = 0u;
    {
        const uint32_t q = lane < c0 ? 0u : (lane < c0 + c1n ? 1u : 2u);
        const uint32_t r = lane - (q == 0u ? 0u : (q == 1u ? c0 : c0 + c1n));
        const uint64_t bits = q == 0u ? m0 : (q == 1u ? m1 : m2);
        pos = active ? 64u * q + select_bit(bits, r) : 0u;
    }
    Region g;
    g.active = active;
    const int px = (int)pos % kReg, py = (int)pos / kReg;
    g.px = px;
    g.py = py;
    g.gx = bx0 + px;
    g.gy = by0 + py;
    // lane holding block position p (valid where p is a non-empty position)
    auto lane_of = [&](int p, bool &ok) -> uint32_t {
        const int q = p >> 6, b = p & 63;
        const uint64_t mq = q == 0 ? m0 : (q == 1 ? m1 : m2);
        ok = ok && ((mq >> b) & 1ull) != 0ull;
        const uint32_t before = (uint32_t)__builtin_popcountll(mq & ((1ull << b) - 1ull));
        return before + (q >= 1 ? c0 : 0u) + (q >= 2 ? c1n : 0u);
    };
    const int dx[kDirs] = {0, 0, -1, 1, 1, -1}, dy[kDirs] = {-1, 1, 0, 0, -1, 1};
#pragma unroll
    for (int d = 0; d < kDirs; ++d) {
        const int qx = px + dx[d], qy = py + dy[d];
        bool ok = active && qx >= 0 && qx < kReg && qy >= 0 && qy < kReg;
        const uint32_t l = lane_of(ok ? qy * kReg + qx : 0, ok);
        g.ok[d] = ok;
        g.lane[d] = ok ? l : lane;
    }
    return g;
}

} // namespace blk

} // namespace fractal

