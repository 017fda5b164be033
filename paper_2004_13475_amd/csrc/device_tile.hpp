// device_tile.hpp -- one rho x rho tile of a gasket step on gfx950.
//
// A workgroup stages the tile plus a one-cell halo of the input state in LDS,
// then every lane computes whole 4/8/16-byte chunks of output rows and writes
// them back with one vector store per chunk.  Only chunks that contain a
// gasket member are read or written: off-gasket cells are 0 in both buffers
// by contract, so a chunk without members is 0 on input and stays 0.
// The fused form advances T steps per launch: it stages T halo rows and one
// extra 16-byte chunk column on each side, runs the T-1 intermediate steps
// between two LDS buffers over that whole region (cells near its edge go
// wrong, but the damage moves inward one cell per step and T is at most the
// cells of one chunk, so it never reaches the tile), and computes the last
// step on the tile itself: T steps for one read and one write of the state.
//
// One-step LDS row layout (bytes): cell x0 + dx of a staged row sits at byte
// 16 + dx * S for dx in [-1, rho + 1); for uint8 tiles narrower than a word
// the right halo cell sits directly after the tile bytes.  Rows 0 and
// rho + 1 are the halo rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fractal {

enum : int { RULE_CA = 0, RULE_HEAT = 1 };

template <int RULE, int R>
struct Geom {
    static constexpr int S = (RULE == RULE_CA) ? 1 : 4;      // bytes per cell
    static constexpr int RHO = 1 << R;                        // tile side
    static constexpr int RB = RHO * S;                        // tile row bytes
    static constexpr int CB = RB >= 16 ? 16 : (RB >= 8 ? 8 : 4); // chunk bytes
    static constexpr int W = CB / 4;                          // words per chunk
    static constexpr bool TINY = RB < 4;                      // u8, rho <= 2
    static constexpr int CPR = TINY ? 1 : RB / CB;            // chunks per row
    static constexpr int CCELLS = TINY ? RHO : CB / S;        // cells per chunk
    static constexpr int CLOG = TINY ? R : (S == 1 ? (CB == 16 ? 4 : (CB == 8 ? 3 : 2))
                                                   : (CB == 16 ? 2 : (CB == 8 ? 1 : 0)));
    static constexpr int OFF = 16;                            // tile byte offset
    static constexpr int PITCH = OFF + CPR * CB + 16;         // LDS row bytes
    static constexpr int ROWS = RHO + 2;
    static constexpr int SPARE = ROWS * PITCH;               // sink for idle lanes
    static constexpr int LDS_BYTES = SPARE + 16;
    // the fused form needs whole 16-byte chunks per row
    static constexpr bool FUSABLE = RB >= 16;
    static constexpr int OFFW = OFF / 4;
    static constexpr int PITCHW = PITCH / 4;
    static constexpr int RIGHTW = OFFW + CPR * W;             // right halo word
    // 64-byte row segments: log2 of the cells in one segment
    static constexpr int SEGLOG = S == 1 ? 6 : 4;
    static constexpr int SLOG = SEGLOG > CLOG ? SEGLOG : CLOG;
};

// Launch-variant flags of the tile engine.
enum : int {
    TILE_SEGMENTS = 1, // read and write whole 64-byte segments that hold a
                       // member (chunks of them without members carry 0s)
    TILE_NT_STORE = 2, // non-temporal hint on output stores
    TILE_FUSE2 = 8,    // two steps per launch (tiles with rows of >= 16 bytes)
    TILE_FUSE4 = 16,   // four steps per launch (same condition)
};

template <int FL>
constexpr int fused_steps()
{
    return (FL & TILE_FUSE4) ? 4 : ((FL & TILE_FUSE2) ? 2 : 1);
}

// Layout of the fused form: chunk columns -1 .. CPR (column c at byte
// OFF + (c + 1) * CB), a zero guard word on either side, RHO + 2T rows, two
// buffers.
template <int RULE, int R, int T>
struct FGeom {
    using G = Geom<RULE, R>;
    static constexpr int NC = G::CPR + 2;
    static constexpr int OFF = 16;
    static constexpr int PITCH = OFF + NC * G::CB + 16;
    static constexpr int PITCHW = PITCH / 4;
    static constexpr int B0W = (OFF + G::CB) / 4; // word of tile chunk 0
    static constexpr int ROWS = G::RHO + 2 * T;
    static constexpr int BUF = ROWS * PITCH;
    static constexpr int SPARE = 2 * BUF;
    static constexpr int LDS_BYTES = SPARE + 16;
};

template <int BYTES>
struct VecT;
template <>
struct VecT<16> {
    using T = uint4;
};
template <>
struct VecT<8> {
    using T = uint2;
};
template <>
struct VecT<4> {
    using T = uint32_t;
};

// Buffer resources.  A raw buffer access whose offset is at or beyond the
// resource's byte count returns 0 (loads) or is dropped (stores) without
// touching memory; predicated-off chunks use that instead of a branch, so a
// lane can keep all of its loads in flight.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOff = 0x80000000u; // an offset beyond every resource here
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer, 32-bit data format

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

template <int BYTES>
__device__ __forceinline__ typename VecT<BYTES>::T buf_load(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ uint4 buf_load<16>(rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return uint4{v[0], v[1], v[2], v[3]};
}
template <>
__device__ __forceinline__ uint2 buf_load<8>(rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return uint2{v[0], v[1]};
}
template <>
__device__ __forceinline__ uint32_t buf_load<4>(rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// AUX is the instruction's cache-policy field (0 = default; 2 = the
// non-temporal hint, for output that is not read again by this launch).
template <int BYTES, int AUX>
__device__ __forceinline__ void buf_store(rsrc_t r, uint32_t off, const typename VecT<BYTES>::T &v)
{
    if constexpr (BYTES == 16) {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        const u4 d = {v.x, v.y, v.z, v.w};
        __builtin_amdgcn_raw_buffer_store_b128(d, r, off, 0, AUX);
    } else if constexpr (BYTES == 8) {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        const u2 d = {v.x, v.y};
        __builtin_amdgcn_raw_buffer_store_b64(d, r, off, 0, AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, AUX);
    }
}

template <int N>
__device__ __forceinline__ void unpack(const typename VecT<4 * N>::T &v, uint32_t (&w)[N]);
template <>
__device__ __forceinline__ void unpack<4>(const uint4 &v, uint32_t (&w)[4])
{
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
}
template <>
__device__ __forceinline__ void unpack<2>(const uint2 &v, uint32_t (&w)[2])
{
    w[0] = v.x; w[1] = v.y;
}
template <>
__device__ __forceinline__ void unpack<1>(const uint32_t &v, uint32_t (&w)[1])
{
    w[0] = v;
}

template <int N>
__device__ __forceinline__ typename VecT<4 * N>::T pack(const uint32_t (&w)[N]);
template <>
__device__ __forceinline__ uint4 pack<4>(const uint32_t (&w)[4])
{
    return uint4{w[0], w[1], w[2], w[3]};
}
template <>
__device__ __forceinline__ uint2 pack<2>(const uint32_t (&w)[2])
{
    return uint2{w[0], w[1]};
}
template <>
__device__ __forceinline__ uint32_t pack<1>(const uint32_t (&w)[1])
{
    return w[0];
}

// Per-byte test t == K for bytes holding values 0..15: y = t ^ K is zero iff
// equal; y + 15 reaches 16 (bit 4 of the byte) iff y != 0, with no carry
// between bytes.  Returns 0x01 in each equal byte.
template <uint32_t K>
__device__ __forceinline__ uint32_t bytes_eq(uint32_t t)
{
    const uint32_t y = t ^ (K * 0x01010101u);
    return (((y + 0x0F0F0F0Fu) >> 4) & 0x01010101u) ^ 0x01010101u;
}

// Gasket membership of the 4 cells x..x+3 (x a multiple of 4) of row y as
// 0/1 bytes: the word is on the gasket at all iff ((x>>2) & (y>>2)) == 0, and
// then cell x+b is a member iff (b & (y & 3)) == 0.
__device__ __forceinline__ uint32_t member_bytes(uint32_t x, uint32_t y)
{
    // bit 0 of y clears bytes 1 and 3, bit 1 clears bytes 2 and 3
    const uint32_t m = ~((y & 1u) * 0xFF00FF00u) & ~(((y >> 1) & 1u) * 0xFFFF0000u);
    const uint32_t p = 0x01010101u & m;
    return (((x >> 2) & (y >> 2)) == 0u) ? p : 0u;
}

// Heat update of one member cell: (1 - 4a) c + a ((N + S) + (W + E)), with a
// fixed rounding sequence so every kernel that uses it agrees bit for bit.
__device__ __forceinline__ float heat_cell(float c, float up, float dn, float w,
                                           float e, float alpha, float c1)
{
#pragma clang fp contract(off)
    const float s = (up + dn) + (w + e);
    return __builtin_fmaf(alpha, s, c1 * c);
}

struct StepParams {
    const uint8_t *src; // state read by this step
    uint8_t *dst;       // state written by this step
    int k;              // level: n = 2^k
    float alpha;        // heat coefficient
};

// Stage rows y0-1 .. y0+RHO and columns x0-1 .. x0+RHO of the input into LDS
// (cells outside the array or off the gasket read as 0).  Every load of this
// thread is issued before its first LDS write.
template <int RULE, int R, int NT, int FL>
__device__ __forceinline__ void stage_tile(uint8_t *lds, const StepParams &p, uint32_t x0,
                                           uint32_t y0)
{
    using G = Geom<RULE, R>;
    constexpr int PLOG = (FL & TILE_SEGMENTS) ? G::SLOG : G::CLOG;
    using V = typename VecT<G::CB>::T;
    const uint32_t n = 1u << p.k;
    const uint32_t pitch = n * G::S; // bytes per state row (<= 2^18)
    const uint32_t tid = threadIdx.x;
    // resource based at row y0 - 1 (possibly before the buffer; that row is
    // then never addressed), spanning the staged rows
    const rsrc_t src = make_rsrc(p.src + ((int64_t)y0 - 1) * (int64_t)pitch,
                                 (uint32_t)G::ROWS * pitch);
    constexpr int NCHUNK = G::ROWS * G::CPR;
    constexpr int NIT = (NCHUNK + NT - 1) / NT;
    constexpr int NHALO = 2 * G::ROWS;
    constexpr int NHIT = (NHALO + NT - 1) / NT;
    using LV = typename std::conditional<G::TINY, uint32_t, V>::type;
    LV vals[NIT];
    uint32_t hvals[NHIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it / G::CPR, c = it % G::CPR;
        const int64_t y = (int64_t)y0 - 1 + ry;
        const uint32_t xc = x0 + (uint32_t)c * G::CCELLS;
        const bool rowok = it < NCHUNK && y >= 0 && y < (int64_t)n;
        const bool live = rowok && (((xc >> PLOG) & ((uint32_t)y >> PLOG)) == 0u);
        const uint32_t roff = (uint32_t)ry * pitch;
        if constexpr (G::TINY) {
            // rho <= 2 uint8 tile: one word = tile cells, right halo, zeros
            uint32_t word = 0u;
#pragma unroll
            for (int i = 0; i < G::RHO; ++i)
                word |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(
                            src, live ? roff + xc + (uint32_t)i : kOff, 0, 0)
                        << (8 * i);
            const uint32_t xr = x0 + G::RHO;
            const bool hr = rowok && xr < n && ((xr & (uint32_t)y) == 0u);
            word |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(src, hr ? roff + xr : kOff, 0, 0)
                    << (8 * G::RHO);
            vals[q] = word;
        } else {
            vals[q] = buf_load<G::CB>(src, live ? roff + xc * G::S : kOff);
        }
    }
    // halo columns: item 2*ry is cell x0-1, item 2*ry+1 cell x0+rho
#pragma unroll
    for (int q = 0; q < NHIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it >> 1;
        const bool right = it & 1;
        const int64_t y = (int64_t)y0 - 1 + ry;
        const int64_t x = right ? (int64_t)x0 + G::RHO : (int64_t)x0 - 1;
        const bool want = it < NHALO && !(right && G::TINY) && x >= 0 && x < (int64_t)n &&
                          y >= 0 && y < (int64_t)n && ((((uint32_t)x) & (uint32_t)y) == 0u);
        const uint32_t off = want ? (uint32_t)ry * pitch + (uint32_t)x * G::S : kOff;
        if constexpr (G::S == 1) {
            const uint32_t b = __builtin_amdgcn_raw_buffer_load_b8(src, off, 0, 0);
            hvals[q] = right ? b : (b << 24);
        } else {
            hvals[q] = __builtin_amdgcn_raw_buffer_load_b32(src, off, 0, 0);
        }
    }
    // LDS writes are unconditional (idle lanes write a spare slot) so that
    // the loads above are not sunk into a branch.
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it / G::CPR, c = it % G::CPR;
        const int slot = (NCHUNK % NT == 0 || it < NCHUNK) ? ry * G::PITCH + G::OFF + c * G::CB
                                                          : G::SPARE;
        *reinterpret_cast<LV *>(lds + slot) = vals[q];
    }
#pragma unroll
    for (int q = 0; q < NHIT; ++q) {
        const int it = (int)tid + q * NT;
        const int slot = (NHALO % NT == 0 || it < NHALO)
                             ? (it >> 1) * G::PITCH + 4 * ((it & 1) ? G::RIGHTW : G::OFFW - 1)
                             : G::SPARE;
        *reinterpret_cast<uint32_t *>(lds + slot) = hvals[q];
    }
}

// New value of the output chunk whose first word is `base` in LDS row `rmd`
// (rows rmd-1 and rmd+1 above and below, PW words per row), for global row
// y and first cell xc, masked to gasket members.
template <int RULE, int R, int PW>
__device__ __forceinline__ void chunk_update(const uint32_t *lw, int rmd, int base, uint32_t xc,
                                             uint32_t y, float alpha, float c1,
                                             uint32_t (&out)[Geom<RULE, R>::W])
{
    using G = Geom<RULE, R>;
    using V = typename VecT<G::CB>::T;
    const int r_up = (rmd - 1) * PW, r_md = rmd * PW, r_dn = (rmd + 1) * PW;
    uint32_t up[G::W], md[G::W], dn[G::W];
    unpack<G::W>(*reinterpret_cast<const V *>(lw + r_up + base), up);
    unpack<G::W>(*reinterpret_cast<const V *>(lw + r_md + base), md);
    unpack<G::W>(*reinterpret_cast<const V *>(lw + r_dn + base), dn);
    if constexpr (RULE == RULE_CA) {
        const uint32_t vl = lw[r_up + base - 1] + lw[r_md + base - 1] + lw[r_dn + base - 1];
        const uint32_t vr = lw[r_up + base + G::W] + lw[r_md + base + G::W] + lw[r_dn + base + G::W];
        uint32_t vc[G::W];
#pragma unroll
        for (int w = 0; w < G::W; ++w)
            vc[w] = up[w] + md[w] + dn[w]; // column sums, <= 3 per byte
#pragma unroll
        for (int w = 0; w < G::W; ++w) {
            const uint32_t left = (w == 0) ? vl : vc[w - 1];
            const uint32_t right = (w == G::W - 1) ? vr : vc[w + 1];
            // 3x3 sums (centre included), <= 9 per byte, no carries
            const uint32_t t = vc[w] + __builtin_amdgcn_alignbyte(vc[w], left, 3) +
                               __builtin_amdgcn_alignbyte(right, vc[w], 1);
            // B3/S23 with t = count + self: alive iff t == 3, or t == 4 and
            // alive now
            const uint32_t alive = bytes_eq<3>(t) | (md[w] & bytes_eq<4>(t));
            out[w] = G::TINY ? alive : (alive & member_bytes(xc + 4u * (uint32_t)w, y));
        }
    } else {
        const float ml = __uint_as_float(lw[r_md + base - 1]);
        const float mr = __uint_as_float(lw[r_md + base + G::W]);
#pragma unroll
        for (int w = 0; w < G::W; ++w) {
            const float wv = (w == 0) ? ml : __uint_as_float(md[w - 1]);
            const float ev = (w == G::W - 1) ? mr : __uint_as_float(md[w + 1]);
            const float v = heat_cell(__uint_as_float(md[w]), __uint_as_float(up[w]),
                                      __uint_as_float(dn[w]), wv, ev, alpha, c1);
            const uint32_t x = xc + (uint32_t)w;
            out[w] = ((x & y) == 0u) ? __float_as_uint(v) : 0u;
        }
    }
}

// Compute the tile's rows from an LDS buffer (PW words per row, tile row j
// in LDS row j + ROW0, tile chunk 0 starting at word B0W) and store the
// chunks that hold a member.
template <int RULE, int R, int NT, int FL, int PW, int B0W, int ROW0>
__device__ __forceinline__ void store_tile(const uint8_t *lds, const StepParams &p, uint32_t x0,
                                           uint32_t y0)
{
    using G = Geom<RULE, R>;
    using V = typename VecT<G::CB>::T;
    constexpr int PLOG = (FL & TILE_SEGMENTS) ? G::SLOG : G::CLOG;
    constexpr int AUX = (FL & TILE_NT_STORE) ? 2 : 0;
    const uint32_t pitch = (1u << p.k) * G::S;
    const uint32_t tid = threadIdx.x;
    const rsrc_t dst = make_rsrc(p.dst + (size_t)y0 * pitch, (uint32_t)G::RHO * pitch);
    const float alpha = p.alpha;
    const float c1 = 1.0f - 4.0f * alpha;
    const uint32_t *lw = reinterpret_cast<const uint32_t *>(lds);
    constexpr int NOUT = G::RHO * G::CPR;
#pragma unroll
    for (int q = 0; q < (NOUT + NT - 1) / NT; ++q) {
        const int it = (int)tid + q * NT;
        if (NOUT % NT != 0 && it >= NOUT)
            break;
        const int j = it / G::CPR, c = it % G::CPR;
        const uint32_t y = y0 + (uint32_t)j;
        const uint32_t xc = x0 + (uint32_t)c * G::CCELLS;
        const uint32_t ooff = (uint32_t)j * pitch + xc * G::S;
        if (((xc >> G::CLOG) & (y >> G::CLOG)) != 0u) {
            // no member in this chunk: it is 0 and stays 0; with whole
            // segments it is rewritten as 0 when its segment holds a member
            if constexpr (PLOG != G::CLOG && !G::TINY) {
                if (((xc >> PLOG) & (y >> PLOG)) == 0u)
                    buf_store<G::CB, AUX>(dst, ooff, V{});
            }
            continue;
        }
        uint32_t out[G::W];
        chunk_update<RULE, R, PW>(lw, j + ROW0, B0W + c * G::W, xc, y, alpha, c1, out);
        if constexpr (G::TINY) {
            // x0 is not word-aligned here: mask and store each cell on its own
#pragma unroll
            for (int i = 0; i < G::RHO; ++i) {
                const uint8_t b = (((xc + (uint32_t)i) & y) == 0u) ? (uint8_t)((out[0] >> (8 * i)) & 1u)
                                                                   : (uint8_t)0;
                __builtin_amdgcn_raw_buffer_store_b8(b, dst, ooff + (uint32_t)i, 0, AUX);
            }
        } else {
            buf_store<G::CB, AUX>(dst, ooff, pack<G::W>(out));
        }
    }
}

// Fused form, staging: rows y0-T .. y0+rho+T-1, chunk columns -1 .. CPR of
// the input into buffer 0 (cells outside the array or in segments without
// members read as 0), and zero guard words in both buffers.
template <int RULE, int R, int NT, int FL, int T>
__device__ __forceinline__ void stage_fused(uint8_t *lds, const StepParams &p, uint32_t x0,
                                            uint32_t y0)
{
    using G = Geom<RULE, R>;
    using FG = FGeom<RULE, R, T>;
    using V = typename VecT<G::CB>::T;
    constexpr int PLOG = (FL & TILE_SEGMENTS) ? G::SLOG : G::CLOG;
    const uint32_t n = 1u << p.k;
    const uint32_t pitch = n * G::S;
    const uint32_t tid = threadIdx.x;
    const rsrc_t src = make_rsrc(p.src + ((int64_t)y0 - T) * (int64_t)pitch,
                                 (uint32_t)FG::ROWS * pitch);
    constexpr int NCHUNK = FG::ROWS * FG::NC;
    constexpr int NIT = (NCHUNK + NT - 1) / NT;
    V vals[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it / FG::NC, c = it % FG::NC - 1;
        const int64_t y = (int64_t)y0 - T + ry;
        const int64_t xc = (int64_t)x0 + (int64_t)c * G::CCELLS;
        const bool ok = it < NCHUNK && y >= 0 && y < (int64_t)n && xc >= 0 && xc < (int64_t)n &&
                        ((((uint32_t)xc >> PLOG) & ((uint32_t)y >> PLOG)) == 0u);
        vals[q] = buf_load<G::CB>(src, ok ? (uint32_t)ry * pitch + (uint32_t)xc * G::S : kOff);
    }
    for (int it = (int)tid; it < FG::ROWS; it += NT) {
        uint32_t *row = reinterpret_cast<uint32_t *>(lds + it * FG::PITCH);
        row[FG::OFF / 4 - 1] = 0u;
        row[(FG::OFF + FG::NC * G::CB) / 4] = 0u;
        row += FG::BUF / 4;
        row[FG::OFF / 4 - 1] = 0u;
        row[(FG::OFF + FG::NC * G::CB) / 4] = 0u;
    }
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it / FG::NC, c = it % FG::NC;
        const int slot = (NCHUNK % NT == 0 || it < NCHUNK) ? ry * FG::PITCH + FG::OFF + c * G::CB
                                                          : FG::SPARE;
        *reinterpret_cast<V *>(lds + slot) = vals[q];
    }
}

// Fused form, intermediate step t (1 <= t < T): from the buffer holding step
// t-1 into the other one, rows t .. rho+2T-1-t, every chunk column.  Cells
// outside the array and chunks without members are written as 0.
template <int RULE, int R, int NT, int T>
__device__ __forceinline__ void fused_step(uint8_t *lds, const StepParams &p, uint32_t x0,
                                           uint32_t y0, int t)
{
    using G = Geom<RULE, R>;
    using FG = FGeom<RULE, R, T>;
    using V = typename VecT<G::CB>::T;
    const uint32_t n = 1u << p.k;
    const float alpha = p.alpha;
    const float c1 = 1.0f - 4.0f * alpha;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(lds + ((t - 1) & 1) * FG::BUF);
    uint8_t *dst = lds + (t & 1) * FG::BUF;
    const int rows = FG::ROWS - 2 * t;
    const int items = rows * FG::NC;
    for (int it = (int)threadIdx.x; it < items; it += NT) {
        const int ry = t + it / FG::NC, c = it % FG::NC - 1;
        const int64_t y = (int64_t)y0 - T + ry;
        const int64_t xc = (int64_t)x0 + (int64_t)c * G::CCELLS;
        uint32_t out[G::W];
        if (y < 0 || y >= (int64_t)n || xc < 0 || xc >= (int64_t)n ||
            ((((uint32_t)xc >> G::CLOG) & ((uint32_t)y >> G::CLOG)) != 0u)) {
            // 0 in the staged buffer already, and in the other one from
            // step 1 on
            if (t > 1)
                continue;
#pragma unroll
            for (int w = 0; w < G::W; ++w)
                out[w] = 0u;
        } else {
            chunk_update<RULE, R, FG::PITCHW>(src, ry, FG::B0W + c * G::W, (uint32_t)xc,
                                              (uint32_t)y, alpha, c1, out);
        }
        *reinterpret_cast<V *>(dst + ry * FG::PITCH + FG::OFF + (c + 1) * G::CB) = pack<G::W>(out);
    }
}

// Process the tile whose top-left cell is (x0, y0): one step, or T steps
// with a fused flag.  All NT threads of the workgroup must call it (it
// contains workgroup barriers).
template <int RULE, int R, int NT, int FL = 0>
__device__ __forceinline__ void tile_step(uint8_t *lds, const StepParams &p,
                                          uint32_t x0, uint32_t y0)
{
    using G = Geom<RULE, R>;
    constexpr int T = fused_steps<FL>();
    if constexpr (T > 1 && G::FUSABLE) {
        using FG = FGeom<RULE, R, T>;
        stage_fused<RULE, R, NT, FL, T>(lds, p, x0, y0);
        __syncthreads();
#pragma unroll
        for (int t = 1; t < T; ++t) {
            fused_step<RULE, R, NT, T>(lds, p, x0, y0, t);
            __syncthreads();
        }
        store_tile<RULE, R, NT, FL, FG::PITCHW, FG::B0W, T>(lds + ((T - 1) & 1) * FG::BUF, p, x0,
                                                            y0);
    } else {
        stage_tile<RULE, R, NT, FL>(lds, p, x0, y0);
        __syncthreads();
        store_tile<RULE, R, NT, FL, G::PITCHW, G::OFFW, 1>(lds, p, x0, y0);
    }
}

// LDS bytes a step kernel of this shape needs.
template <int RULE, int R, int FL>
constexpr int tile_lds_bytes()
{
    return (fused_steps<FL>() > 1 && Geom<RULE, R>::FUSABLE)
               ? FGeom<RULE, R, fused_steps<FL>()>::LDS_BYTES
               : Geom<RULE, R>::LDS_BYTES;
}

} // namespace fractal
