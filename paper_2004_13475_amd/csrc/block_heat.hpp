// block_heat.hpp -- the block engine of the float32 heat step: one
// wavefront per 64 x 64 tile, one lane per non-empty 8 x 8 block.
//
// A tile of a level-k gasket is a level-3 gasket of 8 x 8 blocks, and its
// halo of 16 cells (two blocks on each side) holds more non-empty blocks of
// the neighbouring tiles: at most 54 in the 12 x 12 blocks of the region,
// so one block per lane fits one wavefront.  Lanes take the region's
// non-empty blocks in row-major order, keep the 27 member cells of their
// block in registers for the whole launch, and exchange across block edges
// by ds_bpermute: in a gasket only the corner cells of two side-by-side
// blocks touch (the cell at (0,0) of a block and the one at (0,7) of the
// block above it, (7,0) of the block to its left), so a step needs four
// values from other lanes.  No LDS, no barrier.  Blocks near the region's
// edge see zeros for what lies outside it; the damage moves one cell per
// step and the tile is 16 cells in, so a launch of up to 16 steps leaves the
// tile exact.  The arithmetic per cell is the march and LDS engines'
// (fma(a, (N + S) + (W + E), (1 - 4a) u), neighbours that cannot be members
// left out), so all engines agree bit for bit on non-negative states.  Work
// goes only to non-empty blocks: where the march walks every 16-byte chunk
// of a tile's bounding box (a third of them hold a member in a 64 x 64
// float32 tile), here 27 of the 64 cells of each active lane's block are
// members and 16 of 64 lanes idle at most.
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

__device__ __forceinline__ float pull(uint32_t lane, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute((int)(lane << 2), __float_as_int(v)));
}

// a + b over the terms present (at least one is)
template <bool A, bool B>
__device__ __forceinline__ float sum2(float a, float b)
{
#pragma clang fp contract(off)
    if constexpr (A && B)
        return a + b;
    else if constexpr (A)
        return a;
    else
        return b;
}

struct Cells {
    float v[kBlk][kBlk]; // v[j][i]: cell (i, j); only members are used
};

// One step of the block's members: in -> out.  nN, nS, nW, nE: the north
// block's (0,7), the south block's (0,0), the west block's (7,0) and the
// east block's (0,0) (0 where there is none).
__device__ __forceinline__ void block_step(const Cells &in, Cells &out, float nN, float nS,
                                           float nW, float nE, float alpha, float c1)
{
    static_for<0, kBlk>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        static_for<0, kBlk>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (mem(i, j)) {
                // neighbours inside the block, or the one cross-block value
                // (only corner cells touch the next block)
                constexpr bool HU = j > 0 ? mem(i, j - 1) : i == 0;
                constexpr bool HD = j < kBlk - 1 ? mem(i, j + 1) : i == 0;
                constexpr bool HW = i > 0 ? mem(i - 1, j) : j == 0;
                constexpr bool HE = i < kBlk - 1 ? mem(i + 1, j) : j == 0;
                static_assert(HU || HD || HW || HE, "a member has a member neighbour");
                const float up = j > 0 ? in.v[j > 0 ? j - 1 : 0][i] : nN;
                const float dn = j < kBlk - 1 ? in.v[j < kBlk - 1 ? j + 1 : 0][i] : nS;
                const float wv = i > 0 ? in.v[j][i > 0 ? i - 1 : 0] : nW;
                const float ev = i < kBlk - 1 ? in.v[j][i < kBlk - 1 ? i + 1 : 0] : nE;
                float sum;
                {
#pragma clang fp contract(off)
                    if constexpr ((HU || HD) && (HW || HE))
                        sum = sum2<HU, HD>(up, dn) + sum2<HW, HE>(wv, ev);
                    else if constexpr (HU || HD)
                        sum = sum2<HU, HD>(up, dn);
                    else
                        sum = sum2<HW, HE>(wv, ev);
                    out.v[j][i] = __builtin_fmaf(alpha, sum, c1 * in.v[j][i]);
                }
            } else {
                out.v[j][i] = 0.0f;
            }
        });
    });
}

} // namespace blk

// One wavefront advances the tile t of a level-k state `steps` steps
// (1..16), src -> dst; all 64 lanes call it.
template <int FL>
__device__ __forceinline__ void block_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                           float alpha_in, TileXY t, int steps)
{
    using namespace blk;
    const uint32_t lane = lane_id();
    // the region's non-empty blocks, in row-major order of the 12 x 12
    // positions (three ballots of 64 positions)
    const int nbl = 1 << (k - 3); // blocks per array side
    const int bx0 = (int)(t.x << (kTileLog - 3)) - kHaloBlk;
    const int by0 = (int)(t.y << (kTileLog - 3)) - kHaloBlk;
    uint64_t m[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int p = (int)lane + 64 * q;
        const int gx = bx0 + p % kReg, gy = by0 + p / kReg;
        const bool ne = p < kPos && gx >= 0 && gy >= 0 && gx < nbl && gy < nbl && (gx & gy) == 0;
        m[q] = __builtin_amdgcn_ballot_w64(ne);
    }
    const uint32_t c0 = (uint32_t)__builtin_popcountll(m[0]);
    const uint32_t c1n = (uint32_t)__builtin_popcountll(m[1]);
    const uint32_t nblocks = c0 + c1n + (uint32_t)__builtin_popcountll(m[2]);
    const bool active = lane < nblocks;
    // this lane's block: the lane-th non-empty position
    uint32_t pos = 0u;
    {
        const uint32_t q = lane < c0 ? 0u : (lane < c0 + c1n ? 1u : 2u);
        const uint32_t r = lane - (q == 0u ? 0u : (q == 1u ? c0 : c0 + c1n));
        const uint64_t bits = q == 0u ? m[0] : (q == 1u ? m[1] : m[2]);
        pos = active ? 64u * q + select_bit(bits, r) : 0u;
    }
    const int px = (int)pos % kReg, py = (int)pos / kReg;
    // lane holding block position p (valid where p is a non-empty position)
    auto lane_of = [&](int p, bool &ok) -> uint32_t {
        const int q = p >> 6, b = p & 63;
        const uint64_t mq = q == 0 ? m[0] : (q == 1 ? m[1] : m[2]);
        ok = ok && ((mq >> b) & 1ull) != 0ull;
        const uint32_t before = (uint32_t)__builtin_popcountll(mq & ((1ull << b) - 1ull));
        return before + (q >= 1 ? c0 : 0u) + (q >= 2 ? c1n : 0u);
    };
    bool okN = active && py > 0, okS = active && py < kReg - 1;
    bool okW = active && px > 0, okE = active && px < kReg - 1;
    uint32_t lN = lane_of(okN ? (int)pos - kReg : 0, okN);
    uint32_t lS = lane_of(okS ? (int)pos + kReg : 0, okS);
    uint32_t lW = lane_of(okW ? (int)pos - 1 : 0, okW);
    uint32_t lE = lane_of(okE ? (int)pos + 1 : 0, okE);
    lN = okN ? lN : lane;
    lS = okS ? lS : lane;
    lW = okW ? lW : lane;
    lE = okE ? lE : lane;

    // load the block's member chunks (rows 4..7 hold members in their
    // first four cells only)
    const int n = 1 << k;
    const int gx = bx0 + px, gy = by0 + py;
    const int64_t base = ((int64_t)(gy * kBlk) * n + (int64_t)gx * kBlk) * 4;
    Cells c;
    {
        using gf4 = const __attribute__((address_space(1))) f32x4;
        const uint8_t *src = src_state + (active ? base : 0);
        static_for<0, kBlk>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const f32x4 v0 = *(gf4 *)(src + (int64_t)j * n * 4);
            const f32x4 v1 = (j & 4) == 0 ? *(gf4 *)(src + (int64_t)j * n * 4 + 16) : f32x4{0, 0, 0, 0};
            static_for<0, 4>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                c.v[j][i] = mem(i, j) ? v0[i] : 0.0f;
                c.v[j][i + 4] = mem(i + 4, j) ? v1[i] : 0.0f;
            });
        });
        if (!active)
            static_for<0, kBlk>([&](auto jc) {
                static_for<0, kBlk>([&](auto ic) { c.v[decltype(jc)::value][decltype(ic)::value] = 0.0f; });
            });
    }

    const float alpha = alpha_in;
    const float c1 = 1.0f - 4.0f * alpha;
    Cells d;
    auto exchange_step = [&](const Cells &in, Cells &out) {
        float nN = pull(lN, in.v[kBlk - 1][0]);
        float nS = pull(lS, in.v[0][0]);
        float nW = pull(lW, in.v[0][kBlk - 1]);
        float nE = pull(lE, in.v[0][0]);
        nN = okN ? nN : 0.0f;
        nS = okS ? nS : 0.0f;
        nW = okW ? nW : 0.0f;
        nE = okE ? nE : 0.0f;
        block_step(in, out, nN, nS, nW, nE, alpha, c1);
    };
    int s = 0;
    for (; s + 2 <= steps; s += 2) {
        exchange_step(c, d);
        exchange_step(d, c);
    }
    if (s < steps) {
        exchange_step(c, d);
        c = d;
    }

    // the tile's own blocks write their rows; a 64-byte segment spans two
    // blocks, so an even block whose right-hand partner is empty writes the
    // partner's half as zeros (whole segments are written)
    const bool inner = active && px >= kHaloBlk && px < kHaloBlk + kTileBlk && py >= kHaloBlk &&
                       py < kHaloBlk + kTileBlk;
    if (inner) {
        uint8_t *dst = dst_state + base;
        const bool zero_partner = (gx & 1) == 0 && ((gx + 1) & gy) != 0;
        static_for<0, kBlk>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            f32x4 v0, v1;
            static_for<0, 4>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                v0[i] = mem(i, j) ? c.v[j][i] : 0.0f;
                v1[i] = mem(i + 4, j) ? c.v[j][i + 4] : 0.0f;
            });
            f32x4 *p = reinterpret_cast<f32x4 *>(dst + (int64_t)j * n * 4);
            const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (FL & TILE_NT_STORE) {
                __builtin_nontemporal_store(v0, p);
                __builtin_nontemporal_store(v1, p + 1);
                if (zero_partner) {
                    __builtin_nontemporal_store(z, p + 2);
                    __builtin_nontemporal_store(z, p + 3);
                }
            } else {
                p[0] = v0;
                p[1] = v1;
                if (zero_partner) {
                    p[2] = z;
                    p[3] = z;
                }
            }
        });
    }
}

} // namespace fractal
