// device_march.hpp -- the register-march form of a tile launch on gfx950:
// T steps per launch with no LDS and no barriers.
//
// A wavefront takes P tiles side by side.  Each tile gets a group of lanes:
// rho * S / 16 interior lanes, each holding one 16-byte chunk of a tile row,
// and HL halo lanes on either side holding the chunks next to the tile.  The
// group walks down a band of the tile's rows, from T rows above the band to T
// rows below it, loading one row per stride of the walk.  Step t of the
// update runs t rows behind the load, entirely in registers: each level
// keeps the two rows before its newest, and the cells left and right of a
// chunk come from the neighbouring lanes by a DPP wave shift.  Cells near a
// group's edges and near the walk's ends go wrong (the halo lanes see the
// next group's data, the first rows see zeros), but the damage moves one cell
// per step and T is at most the halo's width and height, so the band's own
// cells come out exact.  Per cell the arithmetic is the one the LDS tile
// engine uses, so both engines agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_map.hpp"
#include "device_tile.hpp"
#include "internal.hpp"

namespace fractal {

template <int RULE, int R, int T, int HL>
struct MGeom {
    static constexpr int S = (RULE == RULE_CA) ? 1 : 4; // bytes per cell
    static constexpr int RHO = 1 << R;
    static constexpr int CC = 16 / S;                    // cells per lane chunk
    static constexpr int SLOG = (RULE == RULE_CA) ? 6 : 4; // cells per 64-byte segment (log2)
    static constexpr int IL = RHO / CC;                  // interior lanes per tile
    static constexpr int GL = IL + 2 * HL;               // lanes per tile
    static constexpr int P = (IL >= 1 && GL <= 64) ? 64 / GL : 0; // tiles per wavefront
    static constexpr bool VALID = P >= 1 && T >= 1 && T <= HL * CC;
};

// Launch shape of a T-step march: halo lanes per side (T <= HL * cells per
// chunk), the wavefronts per SIMD its register allocation must allow, and
// the rows it loads ahead of the walk -- measured fastest at level 16: eight
// steps keep their 64 words of row state at three wavefronts per SIMD; the
// automaton's 16-cell chunks afford eight rows of prefetch at four steps.
constexpr int march_hl(int rule, int T) { return T <= (rule == RULE_CA ? 16 : 4) ? 1 : 2; }
constexpr int march_wpe(int T) { return T >= 8 ? 3 : 1; }
constexpr int march_depth(int rule, int T) { return (rule == RULE_CA && T <= 4) ? 8 : 4; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Value held by lane - 1 (lane 0 reads 0).
__device__ __forceinline__ uint32_t from_left(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF,
                                                 true);
}

// Value held by lane + 1 (lane 63 reads 0).
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130 /* wave_shl:1 */, 0xF, 0xF,
                                                 true);
}

// One level of the walk: the new value of this lane's chunk of row yy from
// the chunks of rows yy-1 (up), yy (md) and yy+1 (dn) after the previous
// level; `inside` is false for chunks outside the array or off the tile set.
template <int RULE>
__device__ __forceinline__ void march_level(const uint32_t (&up)[4], const uint32_t (&md)[4],
                                            const uint32_t (&dn)[4], int xc, int yy, bool inside,
                                            float alpha, float c1, uint32_t (&out)[4])
{
    if constexpr (RULE == RULE_CA) {
        uint32_t vc[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            vc[w] = up[w] + md[w] + dn[w]; // column sums, <= 3 per byte
        const uint32_t vl = from_left(vc[3]);
        const uint32_t vr = from_right(vc[0]);
        // cells x..x+15 with x a multiple of 16: word w is on the gasket iff
        // ((x/4 + w) & (yy/4)) == 0, and then byte b is a member iff
        // (b & (yy & 3)) == 0
        const uint32_t uy = (uint32_t)yy;
        const uint32_t pat = 0x01010101u & ~((uy & 1u) * 0xFF00FF00u) &
                             ~(((uy >> 1) & 1u) * 0xFFFF0000u);
        const uint32_t xw = (uint32_t)xc >> 2;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t left = (w == 0) ? vl : vc[w - 1];
            const uint32_t right = (w == 3) ? vr : vc[w + 1];
            // 3x3 sums, centre included (<= 9 per byte, no carries)
            const uint32_t t = vc[w] + __builtin_amdgcn_alignbyte(vc[w], left, 3) +
                               __builtin_amdgcn_alignbyte(right, vc[w], 1);
            // live neighbours c = t - self; B3/S23 keeps or makes a cell
            // alive iff (c | self) == 3
            const uint32_t alive = bytes_eq<3>((t - md[w]) | md[w]);
            const bool on = inside && (((xw + (uint32_t)w) & (uy >> 2)) == 0u);
            out[w] = on ? (alive & pat) : 0u;
        }
    } else {
        const float ml = __uint_as_float(from_left(md[3]));
        const float mr = __uint_as_float(from_right(md[0]));
        const uint32_t uy = (uint32_t)yy;
        const bool on = inside && (((uint32_t)xc & uy) == 0u);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float wv = (w == 0) ? ml : __uint_as_float(md[w - 1]);
            const float ev = (w == 3) ? mr : __uint_as_float(md[w + 1]);
            const float v = heat_cell(__uint_as_float(md[w]), __uint_as_float(up[w]),
                                      __uint_as_float(dn[w]), wv, ev, alpha, c1);
            out[w] = (on && (((uint32_t)w & uy) == 0u)) ? __float_as_uint(v) : 0u;
        }
    }
}

// Block coordinates of tile `id` under the lambda map: base-3 digit mu-1 of
// the id (CURVE orders) or of omega_x / omega_y for odd / even mu (NATURAL,
// omega = (id mod gx, id div gx)) is beta_mu; bit mu-1 of x is [beta == 2]
// and of y is [beta == 0] (the mirrored replica table).  Per lane.
__device__ __forceinline__ TileXY lambda_lane(uint32_t id, int rb, int order)
{
    uint32_t a = id, b = 0u;
    if (order == FRACTAL_ORDER_NATURAL) {
        const uint32_t gx = pow3_u32((uint32_t)(rb + 1) / 2u);
        b = id / gx;
        a = id - b * gx;
    }
    uint32_t x = 0u, y = 0u;
    for (int mu = 0; mu < rb; ++mu) {
        uint32_t d;
        if (order == FRACTAL_ORDER_NATURAL && (mu & 1)) {
            const uint32_t q = b / 3u;
            d = b - 3u * q;
            b = q;
        } else {
            const uint32_t q = a / 3u;
            d = a - 3u * q;
            a = q;
        }
        x |= (uint32_t)(d == 2u) << mu;
        y |= (uint32_t)(d == 0u) << mu;
    }
    return TileXY{x, y};
}

// Where a lane of a march wavefront works: its group (tile slot) and chunk
// column relative to the tile (-HL .. IL+HL-1).
template <int RULE, int R, int T, int HL>
struct MarchLane {
    using M = MGeom<RULE, R, T, HL>;
    uint32_t grp;
    int col;
    __device__ __forceinline__ MarchLane()
    {
        const uint32_t lane = lane_id();
        grp = lane / (uint32_t)M::GL;
        col = (int)(lane - grp * (uint32_t)M::GL) - HL;
    }
};

// The walk of one group over band `band` (of 2^band_log) of tile t of a
// level-k state: src -> dst, T steps.  Every argument may differ between
// groups; all 64 lanes must call it (the level updates read neighbouring
// lanes), inactive groups with active = false.
template <int RULE, int R, int T, int HL, int FL, int D>
__device__ __forceinline__ void march_walk(const uint8_t *src, uint8_t *dst, int k, float alpha,
                                           TileXY t, int band, int band_log, bool active, int col)
{
    using M = MGeom<RULE, R, T, HL>;
    const int n = 1 << k;
    const int H = M::RHO >> band_log; // band height
    const int xc = (int)(t.x << R) + col * M::CC;
    const int ybase = (int)(t.y << R) + band * H; // first row of the band
    const bool col_ok = active && xc >= 0 && xc < n;
    const bool interior = col >= 0 && col < M::IL;
    const int64_t pitch = (int64_t)n * M::S;
    const int64_t off0 = ((int64_t)ybase - T) * pitch + (int64_t)xc * M::S;
    const int rows = H + 2 * T;
    const float c1 = 1.0f - 4.0f * alpha;

    auto load_row = [&](int i) -> u32x4 {
        const int y = ybase - T + i;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (i < rows && col_ok && y >= 0 && y < n &&
            ((((uint32_t)xc >> M::SLOG) & ((uint32_t)y >> M::SLOG)) == 0u))
            v = *reinterpret_cast<const u32x4 *>(src + off0 + (int64_t)i * pitch);
        return v;
    };

    uint32_t p2[T][4], p1[T][4]; // per level: rows yy-1 and yy of its newest yy+1
#pragma unroll
    for (int l = 0; l < T; ++l)
#pragma unroll
        for (int w = 0; w < 4; ++w)
            p2[l][w] = p1[l][w] = 0u;
    u32x4 ring[D];
#pragma unroll
    for (int d = 0; d < D; ++d)
        ring[d] = load_row(d);
    for (int i0 = 0; i0 < rows; i0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int i = i0 + d;
            uint32_t cur[4] = {ring[d][0], ring[d][1], ring[d][2], ring[d][3]};
            ring[d] = load_row(i + D);
#pragma unroll
            for (int l = 1; l <= T; ++l) {
                const int yy = ybase - T + i - l; // row of level l
                const bool inside = col_ok && yy >= 0 && yy < n;
                uint32_t out[4];
                march_level<RULE>(p2[l - 1], p1[l - 1], cur, xc, yy, inside, alpha, c1, out);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    p2[l - 1][w] = p1[l - 1][w];
                    p1[l - 1][w] = cur[w];
                    cur[w] = out[w];
                }
            }
            // cur: level T at band row j
            const int j = i - 2 * T;
            const int y = ybase + j;
            if (interior && col_ok && j >= 0 && j < H &&
                ((((uint32_t)xc >> M::SLOG) & ((uint32_t)y >> M::SLOG)) == 0u)) {
                const u32x4 o = {cur[0], cur[1], cur[2], cur[3]};
                u32x4 *dp = reinterpret_cast<u32x4 *>(dst + off0 + (int64_t)(j + T) * pitch);
                if constexpr (FL & TILE_NT_STORE)
                    __builtin_nontemporal_store(o, dp);
                else
                    *dp = o;
            }
        }
    }
}

// One gasket: wavefront w of the grid takes (tile, band) items w*P .. w*P+P-1
// (tiles in the map's id order, bands of a tile adjacent).  D: rows loaded
// ahead of the walk; WPE: wavefronts per SIMD the register allocation must
// allow.
template <int RULE, int R, int T, int HL, int MAP, int FL, int WPE = 1, int D = 4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void march_kernel(MarchArgs a)
{
    using M = MGeom<RULE, R, T, HL>;
    static_assert(M::VALID, "march shape");
    const MarchLane<RULE, R, T, HL> ln;
    uint32_t wg = blockIdx.x;
    if (a.order == FRACTAL_ORDER_CURVE_XCD)
        wg = xcd_chunk(wg, gridDim.x);
    const uint32_t wave = wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t item = (uint64_t)wave * M::P + ln.grp; // (tile, band)
    const uint64_t tile = item >> a.band_log;
    const int band = (int)(item & ((1u << a.band_log) - 1u));
    bool active = ln.grp < (uint32_t)M::P && tile < a.total;
    TileXY t{0u, 0u};
    if (active) {
        if constexpr (MAP == MAP_BB) {
            t.x = (uint32_t)tile & ((1u << a.rb) - 1u);
            t.y = (uint32_t)tile >> a.rb;
            active = (t.x & t.y) == 0u;
        } else {
            t = lambda_lane((uint32_t)tile, a.rb, a.order);
        }
    }
    if (__builtin_amdgcn_ballot_w64(active) == 0u)
        return; // whole wavefront idle (no tile, or only empty BB blocks)
    march_walk<RULE, R, T, HL, FL, D>(a.src, a.dst, a.k, a.alpha, t, band, a.band_log, active,
                                      ln.col);
}

} // namespace fractal
