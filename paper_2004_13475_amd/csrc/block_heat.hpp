// block_heat.hpp -- the block engine of the float32 heat step (one
// wavefront per 64 x 64 tile, one lane per non-empty 8 x 8 block; the
// shared setup is in block_engine.hpp).  Each lane keeps the 27 member
// cells of its block in registers for the whole launch; a step needs four
// values from other lanes: in a gasket the cell at (0,0) of a block touches
// only the cell at (0,7) of the block above it and (7,0) of the block to
// its left.  The arithmetic per cell is the march and LDS engines'
// (fma(a, (N + S) + (W + E), (1 - 4a) u), neighbours that cannot be members
// left out), so all engines agree bit for bit on non-negative states.  Work
// goes only to non-empty blocks: where the march walks every 16-byte chunk
// of a tile's bounding box (a third of them hold a member in a 64 x 64
// float32 tile), here 27 of the 64 cells of each active lane's block are
// members.
#pragma once

#include "block_engine.hpp"

namespace fractal {

namespace blk {

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

// The member cells of the block whose first cell is at src (rows P bytes
// apart; rows 4..7 hold members in their first four cells only); zeros
// where the lane holds no block.
__device__ __forceinline__ Cells load_block(const uint8_t *src, int64_t P, bool active)
{
    Cells c;
    using gf4 = const __attribute__((address_space(1))) f32x4;
    static_for<0, kBlk>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const f32x4 v0 = *(gf4 *)(src + j * P);
        const f32x4 v1 = (j & 4) == 0 ? *(gf4 *)(src + j * P + 16) : f32x4{0, 0, 0, 0};
        static_for<0, 4>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            c.v[j][i] = (active && mem(i, j)) ? v0[i] : 0.0f;
            c.v[j][i + 4] = (active && mem(i + 4, j)) ? v1[i] : 0.0f;
        });
    });
    return c;
}

// Writes block (gx, gy)'s rows at dst; a 64-byte segment spans two blocks,
// so an even block whose right-hand partner is empty writes the partner's
// half as zeros (whole segments are written).
template <int FL>
__device__ __forceinline__ void store_block(uint8_t *dst, int64_t P, int gx, int gy, const Cells &c)
{
    const bool zero_partner = (gx & 1) == 0 && ((gx + 1) & gy) != 0;
    static_for<0, kBlk>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        f32x4 v0, v1;
        static_for<0, 4>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            v0[i] = mem(i, j) ? c.v[j][i] : 0.0f;
            v1[i] = mem(i + 4, j) ? c.v[j][i + 4] : 0.0f;
        });
        f32x4 *p = reinterpret_cast<f32x4 *>(dst + j * P);
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

} // namespace blk

// One wavefront advances the tile t of a level-k state `steps` steps
// (1..D), src -> dst, the cells where `lay` puts them; all 64 lanes call it.
template <int FL, int D, class Layout>
__device__ __forceinline__ void block_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                           float alpha_in, TileXY t, int steps, const Layout &lay)
{
    using namespace blk;
    constexpr int H = halo_blocks(D);
    const Region g = block_region<false, D>(k, t);
    const bool active = g.active;
    const int px = g.px, py = g.py;
    const uint32_t lN = g.lane[DN], lS = g.lane[DS], lW = g.lane[DW], lE = g.lane[DE];

    // load the block's member chunks (rows 4..7 hold members in their
    // first four cells only)
    const int gx = g.gx, gy = g.gy;
    const int64_t base = lay.block_off(gx, gy);
    const int64_t P = lay.pitch(); // bytes between a block's rows
    Cells c = load_block(src_state + (active ? base : 0), P, active);

    const float alpha = alpha_in;
    const float c1 = 1.0f - 4.0f * alpha;
    Cells d;
    auto exchange_step = [&](const Cells &in, Cells &out) {
        // (zero from the zero lane where there is no such block)
        const float nN = pull(lN, in.v[kBlk - 1][0]);
        const float nS = pull(lS, in.v[0][0]);
        const float nW = pull(lW, in.v[0][kBlk - 1]);
        const float nE = pull(lE, in.v[0][0]);
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

    // the tile's own blocks write their rows
    const bool inner = active && px >= H && px < H + kTileBlk && py >= H && py < H + kTileBlk;
    if (inner)
        store_block<FL>(dst_state + base, P, gx, gy, c);
}

// One wavefront advances the 128 x 128 tile t of a level-k state `steps`
// steps (1..36), src -> dst, two blocks per lane; all 64 lanes call it.  A
// step reads each neighbouring block's cell from both slots of the lane
// that holds it and keeps the one of the block's slot.
template <int FL, class Layout>
__device__ __forceinline__ void block2_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                            float alpha, TileXY t, int steps, const Layout &lay)
{
    using namespace blk;
    constexpr int H = halo_blocks(36);
    Slot2 sl[2];
    block_region2<false>(k, t, sl);
    const int64_t P = lay.pitch();
    Cells c[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
        c[s] = load_block(src_state + (sl[s].active ? lay.block_off(sl[s].gx, sl[s].gy) : 0), P,
                          sl[s].active);
    const float c1 = 1.0f - 4.0f * alpha;
    // the value of `v` (per slot) held by list entry q
    auto pull2 = [](uint32_t q, float v0, float v1) {
        const float x0 = pull(q & 63u, v0), x1 = pull(q & 63u, v1);
        return (q & 64u) ? x1 : x0;
    };
    auto exchange_step = [&](const Cells (&in)[2], Cells (&out)[2]) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float nN = pull2(sl[s].nb[DN], in[0].v[kBlk - 1][0], in[1].v[kBlk - 1][0]);
            const float nS = pull2(sl[s].nb[DS], in[0].v[0][0], in[1].v[0][0]);
            const float nW = pull2(sl[s].nb[DW], in[0].v[0][kBlk - 1], in[1].v[0][kBlk - 1]);
            const float nE = pull2(sl[s].nb[DE], in[0].v[0][0], in[1].v[0][0]);
            block_step(in[s], out[s], nN, nS, nW, nE, alpha, c1);
        }
    };
    Cells d[2];
    int st = 0;
    for (; st + 2 <= steps; st += 2) {
        exchange_step(c, d);
        exchange_step(d, c);
    }
    if (st < steps) {
        exchange_step(c, d);
        c[0] = d[0];
        c[1] = d[1];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const bool inner = sl[s].active && sl[s].px >= H && sl[s].px < H + kTile2Blk &&
                           sl[s].py >= H && sl[s].py < H + kTile2Blk;
        if (inner)
            store_block<FL>(dst_state + lay.block_off(sl[s].gx, sl[s].gy), P, sl[s].gx, sl[s].gy,
                            c[s]);
    }
}

// The n x n array form.
template <int FL, int D>
__device__ __forceinline__ void block_tile(const uint8_t *src_state, uint8_t *dst_state, int k,
                                           float alpha_in, TileXY t, int steps)
{
    block_tile<FL, D>(src_state, dst_state, k, alpha_in, t, steps,
                      blk::ArrayLayout{(int64_t)4 << k, 4, t});
}

} // namespace fractal
