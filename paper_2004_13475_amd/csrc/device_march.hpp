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

#include <type_traits>

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
// steps keep their row state at three wavefronts per SIMD (sixteen at two);
// the automaton's 16-cell chunks afford eight rows of prefetch at four steps.
constexpr int march_hl(int rule, int T)
{
    return T <= (rule == RULE_CA ? 16 : 4) ? 1 : (T <= 8 ? 2 : 4);
}
// Step counts a march launch takes: up to 16 for the automaton (one chunk
// of halo); up to 8 for heat, and 10, 12 or 16 on tiles of side >= 16 (four
// halo lanes per side: narrower tiles would be mostly halo).
constexpr bool march_supported(int rule, int T, int R)
{
    return T <= 8 || (T <= 16 && (rule == RULE_CA || R >= 4));
}
constexpr int march_wpe(int T) { return T >= 10 ? 2 : (T >= 8 ? 3 : 1); }
// The other occupancy the autotuner may try for the long launches: 3
// wavefronts per SIMD for the automaton's 16 steps (fewer registers per
// lane), 2 for 8 steps (more registers: room for the row state of the wider
// tiles without spills).
constexpr int march_wpe_alt(int T) { return T >= 16 ? 3 : 2; }
// Launch shapes with a kernel for the other occupancy: 8 steps, or the
// automaton's 16 (heat's 16-step row state, 16 levels of 3 rows of 4
// words, needs the registers of 2 wavefronts per SIMD), tiles of side 16,
// 32 or 64.
constexpr bool march_has_alt(int rule, int T, int R)
{
    return (T == 8 || (T == 16 && rule == RULE_CA)) && R >= 4 && R <= 6;
}
// Rows loaded ahead of the walk: a whole number of them per unrolled pass
// (16 rows for the automaton, 12 for heat).  Heat launches of 8 and 16
// steps keep a whole pass in flight: at 16 x 16 tiles and 8 steps that
// costs a wavefront per SIMD of occupancy (4 -> 3) and still measured 3-10%
// faster than 6 or 4 rows; at 16 steps the 12 rows fit the 2 wavefronts per
// SIMD the row state needs anyway (240 registers).
constexpr int march_depth(int rule, int T)
{
    return rule == RULE_CA ? (T <= 4 ? 8 : 4) : (T >= 8 ? 12 : 4);
}
// Band heights (and so band origins) are multiples of this row period.
constexpr int march_row_period(int rule) { return rule == RULE_CA ? 16 : 4; }
// Whether the walk's first passes leave out the levels not yet needed (about
// T(T+1) of the T(H+2T) level rows of a band of H rows) at the price of
// compiling those passes separately.
constexpr bool march_peel(int /*rule*/, int /*T*/) { return true; }

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

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Row state of one lane chunk (16 cells of memory) and one level of the
// walk for each rule.  A level computes this lane's chunk of row yy from the
// chunks of rows yy-1 (up), yy (md) and yy+1 (dn) of the previous level;
// `ok` is false for chunks outside the array, off the tile set, or whose
// cells (xc & yy) rules off the gasket as a whole; YQ = yy mod Q is known at
// compile time (tile and band origins are multiples of Q and the walk is
// unrolled Q rows at a time), so the member pattern inside the chunk is a
// constant.
template <int RULE>
struct MarchRule;

// Automaton: registers hold cells as 4-bit counters, 8 per word (cell
// xc + 8j + n in bits 4n..4n+3 of word j), so one add sums 8 cells.
template <>
struct MarchRule<RULE_CA> {
    static constexpr int W = 2;  // words per chunk
    static constexpr int Q = 16; // row period of the in-chunk member pattern
    static constexpr int U = 16; // rows per unrolled pass of the walk
    // 16 bytes of 0/1 cells -> nibbles: byte j of a word gets cells 2j
    // (low nibble) and 2j+1 (high nibble)
    static __device__ __forceinline__ void load(const u32x4 &v, uint32_t (&s)[W])
    {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t lo = v[2 * j], hi = v[2 * j + 1];
            const uint32_t ev = __builtin_amdgcn_perm(hi, lo, 0x06040200u); // cells 0,2,4,6
            const uint32_t od = __builtin_amdgcn_perm(hi, lo, 0x07050301u); // cells 1,3,5,7
            s[j] = ev | (od << 4);
        }
    }
    static __device__ __forceinline__ u32x4 store(const uint32_t (&s)[W])
    {
        u32x4 v;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t ev = s[j] & 0x0F0F0F0Fu, od = (s[j] >> 4) & 0x0F0F0F0Fu;
            v[2 * j] = __builtin_amdgcn_perm(od, ev, 0x05010400u);
            v[2 * j + 1] = __builtin_amdgcn_perm(od, ev, 0x07030602u);
        }
        return v;
    }
    // member nibbles (value 1 << 3) of word j for rows with yy mod 16 == YQ:
    // cell 8j + n is a member iff ((8j + n) & YQ) == 0
    template <int YQ>
    static constexpr uint32_t pattern(int j)
    {
        uint32_t p = 0u;
        for (int c = 0; c < 8; ++c)
            if (((8 * j + c) & YQ) == 0)
                p |= 8u << (4 * c);
        return p;
    }
    template <int YQ>
    static __device__ __forceinline__ void level(const uint32_t (&up)[W], const uint32_t (&md)[W],
                                                 const uint32_t (&dn)[W], bool ok, float, float,
                                                 uint32_t (&out)[W])
    {
        uint32_t vc[W];
#pragma unroll
        for (int j = 0; j < W; ++j)
            vc[j] = up[j] + md[j] + dn[j]; // column sums, <= 3 per nibble
        const uint32_t vl = from_left(vc[W - 1]);
        const uint32_t vr = from_right(vc[0]);
        const uint32_t m = ok ? ~0u : 0u;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const uint32_t left = (j == 0) ? vl : vc[j - 1];
            const uint32_t right = (j == W - 1) ? vr : vc[j + 1];
            // 3x3 sums, centre included (<= 9 per nibble, no carries): each
            // nibble plus its west (funnel shift in from the left word) and
            // east neighbours
            const uint32_t t = vc[j] + __builtin_amdgcn_alignbit(vc[j], left, 28) +
                               __builtin_amdgcn_alignbit(right, vc[j], 4);
            // live neighbours c = t - self; B3/S23 keeps or makes a cell
            // alive iff (c | self) == 3; y = that ^ 3 is 0 exactly then, and
            // (y & 7) + 7 reaches bit 3 iff y & 7 != 0 (no carry out)
            const uint32_t y = ((t - md[j]) | md[j]) ^ 0x33333333u;
            const uint32_t h = ((y & 0x77777777u) + 0x77777777u) | y;
            out[j] = ((~h & m) & pattern<YQ>(j)) >> 3;
        }
    }
};

// Heat: registers hold the 4 float32 cells of the chunk.
template <>
struct MarchRule<RULE_HEAT> {
    static constexpr int W = 4;
    static constexpr int Q = 4;
    // a multiple of 3 as well: the three rows each level keeps then rotate
    // through fixed registers, with no moves at the loop's back edge
    static constexpr int U = 12;
    static __device__ __forceinline__ void load(const u32x4 &v, uint32_t (&s)[W])
    {
#pragma unroll
        for (int w = 0; w < W; ++w)
            s[w] = v[w];
    }
    static __device__ __forceinline__ u32x4 store(const uint32_t (&s)[W])
    {
        return u32x4{s[0], s[1], s[2], s[3]};
    }
    // a + b over the terms that are present (at least one is)
    template <bool A, bool B>
    static __device__ __forceinline__ float sum2(float a, float b)
    {
#pragma clang fp contract(off)
        if constexpr (A && B)
            return a + b;
        else if constexpr (A)
            return a;
        else
            return b;
    }
    template <int YQ>
    static __device__ __forceinline__ void level(const uint32_t (&up)[W], const uint32_t (&md)[W],
                                                 const uint32_t (&dn)[W], bool ok, float alpha,
                                                 float c1, uint32_t (&out)[W])
    {
        // Cell w of a chunk in a row of phase p is a member iff (w & p) == 0
        // (given that row's ok).  Neighbours that are off the gasket by phase
        // alone hold 0 and are left out of the sum ((N + S) + (W + E) as in
        // heat_cell; leaving out a +0 term changes at most the sign of a
        // zero).  Where ok is false every cell of the chunk, and of the
        // previous level at the same place, is 0, so a coefficient of 0
        // gives 0 without a select per cell.
        constexpr int PU = (YQ + Q - 1) % Q; // phase of the row above
        constexpr int PD = (YQ + 1) % Q;     // phase of the row below
        const float a = ok ? alpha : 0.0f;
        float ml = 0.0f, mr = 0.0f;
        if constexpr ((3 & YQ) == 0) // cell 3 of the left chunk is a member
            ml = __uint_as_float(from_left(md[3]));
        if constexpr ((3 & YQ) == 0) // cell 3 is a member and needs cell 0 on the right
            mr = __uint_as_float(from_right(md[0]));
        static_for<0, W>([&](auto wc) {
            constexpr int w = decltype(wc)::value;
            if constexpr ((w & YQ) != 0) {
                out[w] = 0u;
            } else {
                constexpr bool HU = (w & PU) == 0, HD = (w & PD) == 0;
                constexpr int WL = (w + 3) & 3, WR = (w + 1) & 3;
                constexpr bool HW = (WL & YQ) == 0, HE = (WR & YQ) == 0;
                static_assert(HU || HD || HW || HE, "a member has a member neighbour");
                const float wv = (w == 0) ? ml : __uint_as_float(md[w == 0 ? 0 : w - 1]);
                const float ev = (w == 3) ? mr : __uint_as_float(md[w == 3 ? 0 : w + 1]);
                float sum;
                {
#pragma clang fp contract(off)
                    if constexpr ((HU || HD) && (HW || HE))
                        sum = sum2<HU, HD>(__uint_as_float(up[w]), __uint_as_float(dn[w])) +
                              sum2<HW, HE>(wv, ev);
                    else if constexpr (HU || HD)
                        sum = sum2<HU, HD>(__uint_as_float(up[w]), __uint_as_float(dn[w]));
                    else
                        sum = sum2<HW, HE>(wv, ev);
                    out[w] = __float_as_uint(__builtin_fmaf(a, sum, c1 * __uint_as_float(md[w])));
                }
            }
        });
    }
};

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

// Where a lane's chunk column of walk row i (array row y) lives, for a
// state stored as the n x n array: `has` tells whether row y has storage,
// `ld` / `st` give the chunk's address in the input / output state.
struct EmbeddedAddr {
    const uint8_t *src;
    uint8_t *dst;
    int64_t off0;  // byte offset of the chunk in walk row 0
    int64_t pitch; // bytes per array row
    int n;
    __device__ __forceinline__ bool has(int y) const { return (uint32_t)y < (uint32_t)n; }
    __device__ __forceinline__ const uint8_t *any() const { return src; }
    __device__ __forceinline__ const uint8_t *ld(int i, int) const
    {
        return src + off0 + (int64_t)i * pitch;
    }
    __device__ __forceinline__ uint8_t *st(int i, int) const
    {
        return dst + off0 + (int64_t)i * pitch;
    }
};

// The walk of one group over the band of H rows starting at array row ybase,
// chunk column starting at array column xc: src -> dst through `A`, T steps.
// Every argument may differ between groups; all 64 lanes must call it (the
// level updates read neighbouring lanes), inactive groups with col_ok false.
template <int RULE, int R, int T, int HL, int FL, int D, bool PEEL = march_peel(RULE, T),
          class Addr>
__device__ __forceinline__ void march_walk_at(const Addr &A, int k, float alpha, int xc,
                                              int ybase, int H, bool col_ok, bool interior)
{
    using M = MGeom<RULE, R, T, HL>;
    using RU = MarchRule<RULE>;
    constexpr int W = RU::W;
    constexpr int Q = RU::Q; // tile and band origins are multiples of Q
    static_assert(Q == march_row_period(RULE), "row period");
    constexpr int U = RU::U;
    static_assert(U % Q == 0 && U % D == 0, "unrolled pass: whole row periods and ring turns");
    const int n = 1 << k;
    const int rows = H + 2 * T;
    const float c1 = 1.0f - 4.0f * alpha;

    // Rows are loaded D rows ahead into a ring.  Every lane loads (a chunk
    // without storage or members reads the always-valid chunk A.any() and
    // is taken as 0 when used): with no branch around the loads the wait
    // for a row can count the loads still in flight.  `take` marks the four
    // words as used at that point, so none of their registers is reused
    // while the load may still write it.
    bool keep[D];
    auto load_row = [&](int i, bool &want) -> u32x4 {
        const int y = ybase - T + i;
        want = i < rows && col_ok && A.has(y) &&
               ((((uint32_t)xc >> M::SLOG) & ((uint32_t)y >> M::SLOG)) == 0u);
        // global memory: a load through a generic pointer would count on
        // the LDS counter as well, whose waits cannot leave loads in flight
        using gu32x4 = const __attribute__((address_space(1))) u32x4;
        return *(gu32x4 *)(want ? A.ld(i, y) : A.any());
    };
    auto take = [](u32x4 v, bool want) -> u32x4 {
        uint32_t a = v[0], b = v[1], c = v[2], e = v[3];
        asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(e));
        return want ? u32x4{a, b, c, e} : u32x4{0u, 0u, 0u, 0u};
    };

    // Per input level, the rows before its newest: with a pass of a whole
    // number of 3 rows, three slots indexed by row mod 3 (no moves at the
    // loop's back edge); otherwise two rows shifted each row.
    constexpr bool RING3 = (U % 3) == 0;
    uint32_t win[T][RING3 ? 3 : 2][W];
#pragma unroll
    for (int l = 0; l < T; ++l)
#pragma unroll
        for (int q = 0; q < (RING3 ? 3 : 2); ++q)
#pragma unroll
            for (int w = 0; w < W; ++w)
                win[l][q][w] = 0u;
    u32x4 ring[D];
#pragma unroll
    for (int d = 0; d < D; ++d)
        ring[d] = load_row(d, keep[d]);
    // One pass of U walk rows from walk row i0.  Level l is needed from the
    // row T - l above the band down, which it reaches at walk row 2l; the
    // first passes (F = i0, known at compile time) leave out the levels not
    // yet needed and keep only their window filling from walk row 2l - 2
    // on; later passes (F < 0) run every level.
    auto pass = [&](int i0, auto fc) {
        constexpr int F = decltype(fc)::value;
        static_for<0, U>([&](auto dc) {
            constexpr int d = decltype(dc)::value;
            const int i = i0 + d;
            uint32_t cur[W];
            RU::load(take(ring[d % D], keep[d % D]), cur);
            ring[d % D] = load_row(i + D, keep[d % D]);
            // keep the prefetch here: the scheduler would otherwise sink it
            // next to its use D rows later under register pressure
            __builtin_amdgcn_sched_barrier(0);
            static_for<1, T + 1>([&](auto lc) {
                constexpr int l = decltype(lc)::value;
                constexpr int yq = (((d - T - l) % Q) + Q) % Q; // (row of level l) mod Q
                if constexpr (F < 0 || F + d >= 2 * l) {
                    const int yy = ybase - T + i - l;
                    const bool ok = col_ok && (uint32_t)yy < (uint32_t)n &&
                                    (((uint32_t)xc & (uint32_t)yy) & ~(uint32_t)(Q - 1)) == 0u;
                    uint32_t out[W];
                    if constexpr (RING3) {
                        // rows i-2, i-1 of level l-1 in slots (i-2) mod 3, (i-1) mod 3
                        RU::template level<yq>(win[l - 1][(d + 1) % 3], win[l - 1][(d + 2) % 3],
                                               cur, ok, alpha, c1, out);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            win[l - 1][d % 3][w] = cur[w];
                            cur[w] = out[w];
                        }
                    } else {
                        RU::template level<yq>(win[l - 1][0], win[l - 1][1], cur, ok, alpha, c1,
                                               out);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            win[l - 1][0][w] = win[l - 1][1][w];
                            win[l - 1][1][w] = cur[w];
                            cur[w] = out[w];
                        }
                    }
                } else if constexpr (F + d >= 2 * l - 2) {
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        if constexpr (RING3) {
                            win[l - 1][d % 3][w] = cur[w];
                        } else {
                            win[l - 1][0][w] = win[l - 1][1][w];
                            win[l - 1][1][w] = cur[w];
                        }
                    }
                }
            });
            // cur: level T at band row j
            if constexpr (F < 0 || F + d >= 2 * T) {
                const int j = i - 2 * T;
                const int y = ybase + j;
                if (interior && col_ok && j >= 0 && j < H &&
                    ((((uint32_t)xc >> M::SLOG) & ((uint32_t)y >> M::SLOG)) == 0u)) {
                    const u32x4 o = RU::store(cur);
                    u32x4 *dp = reinterpret_cast<u32x4 *>(A.st(j + T, y));
                    if constexpr (FL & TILE_NT_STORE)
                        __builtin_nontemporal_store(o, dp);
                    else
                        *dp = o;
                }
            }
        });
    };
    // the first passes start below rows (rows >= 2T + Q > (NP - 1) U);
    // without PEEL every pass runs every level (smaller code)
    constexpr int NP = PEEL ? (2 * T + U - 1) / U : 0;
    static_for<0, NP>([&](auto pc) {
        pass(decltype(pc)::value * U, std::integral_constant<int, decltype(pc)::value * U>{});
    });
    for (int i0 = NP * U; i0 < rows; i0 += U)
        pass(i0, std::integral_constant<int, -1>{});
}

// march_walk_at over the n x n array: rows ybase .. ybase+H-1 of the tile
// column starting at array column x0.
template <int RULE, int R, int T, int HL, int FL, int D, bool PEEL = march_peel(RULE, T)>
__device__ __forceinline__ void march_walk_rows(const uint8_t *src, uint8_t *dst, int k,
                                                float alpha, int x0, int ybase, int H,
                                                bool active, int col)
{
    using M = MGeom<RULE, R, T, HL>;
    const int n = 1 << k;
    const int xc = x0 + col * M::CC;
    EmbeddedAddr A;
    A.src = src;
    A.dst = dst;
    A.pitch = (int64_t)n * M::S;
    A.off0 = ((int64_t)ybase - T) * A.pitch + (int64_t)xc * M::S;
    A.n = n;
    march_walk_at<RULE, R, T, HL, FL, D, PEEL>(A, k, alpha, xc, ybase, H,
                                               active && xc >= 0 && xc < n,
                                               col >= 0 && col < M::IL);
}

// march_walk_at over the n x n array: band `band` (of 2^band_log) of tile t.
template <int RULE, int R, int T, int HL, int FL, int D, bool PEEL = march_peel(RULE, T)>
__device__ __forceinline__ void march_walk(const uint8_t *src, uint8_t *dst, int k, float alpha,
                                           TileXY t, int band, int band_log, bool active, int col)
{
    using M = MGeom<RULE, R, T, HL>;
    const int H = M::RHO >> band_log; // band height, a multiple of the row period
    march_walk_rows<RULE, R, T, HL, FL, D, PEEL>(src, dst, k, alpha, (int)(t.x << R),
                                                 (int)(t.y << R) + band * H, H, active, col);
}

// Vertical stacks of tiles.  In a level-rb gasket of tiles, column tx holds
// the rows ty with (tx & ty) == 0: for tx = 2^j (2v + 1) these are runs of
// 2^j tiles starting at rows 2^(j+1) s with (v & s) == 0, and the columns
// tx = 2^c u hold runs of at least 2^c tiles, starting at rows 2^c s with
// (u & s) == 0.  So the tiles split into classes j = 0 .. c: class j < c is
// a level rb-j-1 gasket of stacks 2^j tiles high and class c a level rb-c
// gasket of stacks 2^c high, each mapped by lambda (Theorem 1 applied to
// the stacks).  A walk down a stack pays the 2T halo rows once for all its
// tiles.  stack_level(j, c, rb) is the gasket level of class j.
__host__ __device__ constexpr int stack_level(int j, int c, int rb)
{
    return j < c ? rb - j - 1 : rb - c;
}

// One gasket: wavefront w of the grid takes (tile, band) items w*P .. w*P+P-1
// (tiles in the map's id order, bands of a tile adjacent), or with stacks
// (lambda map, a.stack_log = c > 0) one class's stacks.  Stack item L of
// class c and the 3^(c-j-1) items from L 3^(c-j-1) of class j < c fill the
// same 2^c x 2^c block of tiles (the low base-3 digits of a curve id pick
// the sub-block), so the grid runs in groups of G = 1 + (3^c - 1) / 2
// wavefronts over P blocks: one wavefront of class c, then 3^(c-j-1) of
// each class j = c-1 .. 0.  Neighbouring tiles of all classes are walked
// close together in time and place (the dies get contiguous runs of groups),
// so halo columns are shared in L2.  D: rows loaded ahead of the walk; WPE:
// wavefronts per SIMD the register allocation must allow.
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
    if (MAP == MAP_LAMBDA && a.stack_log > 0) {
        if (wave >= a.stack_waves)
            return; // past the last group
        const int c = a.stack_log;
        uint32_t pc = 1u; // 3^c
        for (int e = 0; e < c; ++e)
            pc *= 3u;
        const uint32_t G = 1u + (pc - 1u) / 2u;
        const uint32_t g = wave / G, slot = wave - g * G;
        int j = c;
        uint32_t base = 0u, size = 1u; // class j's wavefronts in a group: base .. base+size-1
        if (slot >= 1u) {
            j = c - 1;
            base = 1u;
            while (slot >= base + size) {
                base += size;
                size *= 3u;
                --j;
            }
        }
        const int level = stack_level(j, c, a.rb);
        const uint64_t item = ((uint64_t)g * size + (slot - base)) * M::P + ln.grp;
        uint64_t count = 1u; // stacks in class j: 3^level
        for (int e = 0; e < level; ++e)
            count *= 3u;
        const bool active = ln.grp < (uint32_t)M::P && item < count;
        uint32_t tx = 0u, ty0 = 0u;
        if (active) {
            const TileXY t = lambda_lane((uint32_t)item, level, FRACTAL_ORDER_CURVE);
            tx = j < c ? (2u * t.x + 1u) << j : t.x << c;
            ty0 = j < c ? t.y << (j + 1) : t.y << c;
        }
        if (__builtin_amdgcn_ballot_w64(active) == 0u)
            return;
        march_walk_rows<RULE, R, T, HL, FL, D>(a.src, a.dst, a.k, a.alpha, (int)(tx << R),
                                               (int)(ty0 << R), M::RHO << j, active, ln.col);
        return;
    }
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
