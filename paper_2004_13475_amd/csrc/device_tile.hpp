// device_tile.hpp -- one rho x rho tile of a gasket step on gfx950.
//
// A workgroup stages the tile plus a one-cell halo of the input state in LDS,
// then every lane computes whole 4/8/16-byte chunks of output rows and writes
// them back with one vector store per chunk.  Only chunks that contain a
// gasket member are read or written: off-gasket cells are 0 in both buffers
// by contract, so a chunk without members is 0 on input and stays 0.
// The fused form stages a two-cell halo, computes the intermediate step on
// the tile plus a one-cell ring into a second LDS buffer, and from there the
// final step: two steps for one read and one write of the state.
//
// LDS row layout (bytes): cell x0 + dx of a staged row sits at byte
// 16 + dx * S for dx in [-H, rho + H) (H = halo width); for uint8 tiles
// narrower than a word the right halo cell sits directly after the tile
// bytes.  Rows 0 .. H-1 and the last H rows are the halo rows.
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
    // fused two-step form: RHO + 4 staged rows, then RHO + 2 intermediate rows
    static constexpr bool FUSABLE = RB >= 16;
    static constexpr int ROWS2 = RHO + 4;
    static constexpr int MID = ROWS2 * PITCH;                 // intermediate buffer
    static constexpr int SPARE2 = MID + ROWS * PITCH;
    static constexpr int LDS2_BYTES = SPARE2 + 16;
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

// Stage rows y0-H .. y0+RHO+H-1 and columns x0-H .. x0+RHO+H-1 of the input
// into LDS (cells outside the array or off the gasket read as 0).  Every load
// of this thread is issued before its first LDS write.
template <int RULE, int R, int NT, int FL, int H>
__device__ __forceinline__ void stage_tile(uint8_t *lds, const StepParams &p, uint32_t x0,
                                           uint32_t y0)
{
    using G = Geom<RULE, R>;
    static_assert(H == 1 || (H == 2 && G::FUSABLE), "two-cell halo needs 16-byte rows");
    constexpr int PLOG = (FL & TILE_SEGMENTS) ? G::SLOG : G::CLOG;
    constexpr int NROWS = G::RHO + 2 * H;
    constexpr int SPARE = H == 1 ? G::SPARE : G::SPARE2;
    using V = typename VecT<G::CB>::T;
    const uint32_t n = 1u << p.k;
    const uint32_t pitch = n * G::S; // bytes per state row (<= 2^18)
    const uint32_t tid = threadIdx.x;
    // resource based at row y0 - H (possibly before the buffer; such rows are
    // never addressed), spanning the staged rows
    const rsrc_t src = make_rsrc(p.src + ((int64_t)y0 - H) * (int64_t)pitch,
                                 (uint32_t)NROWS * pitch);
    constexpr int NCHUNK = NROWS * G::CPR;
    constexpr int NIT = (NCHUNK + NT - 1) / NT;
    constexpr int NHALO = 2 * NROWS;
    constexpr int NHIT = (NHALO + NT - 1) / NT;
    using LV = typename std::conditional<G::TINY, uint32_t, V>::type;
    LV vals[NIT];
    uint32_t hvals[NHIT][H];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it / G::CPR, c = it % G::CPR;
        const int64_t y = (int64_t)y0 - H + ry;
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
    // halo columns: item 2*ry is the left run x0-H .. x0-1, item 2*ry+1 the
    // right run x0+rho .. x0+rho+H-1
#pragma unroll
    for (int q = 0; q < NHIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it >> 1;
        const bool right = it & 1;
        const int64_t y = (int64_t)y0 - H + ry;
        const int64_t xa = right ? (int64_t)x0 + G::RHO : (int64_t)x0 - H; // first cell of run
        bool want = it < NHALO && !(right && G::TINY) && xa >= 0 && xa + H <= (int64_t)n &&
                    y >= 0 && y < (int64_t)n;
        if (want) {
            bool anym = false;
#pragma unroll
            for (int h = 0; h < H; ++h)
                anym |= ((((uint32_t)xa + h) & (uint32_t)y) == 0u);
            want = anym;
        }
        const uint32_t off = want ? (uint32_t)ry * pitch + (uint32_t)xa * G::S : kOff;
        if constexpr (G::S == 1) {
            if constexpr (H == 1) {
                const uint32_t b = __builtin_amdgcn_raw_buffer_load_b8(src, off, 0, 0);
                hvals[q][0] = right ? b : (b << 24);
            } else {
                const uint32_t b = __builtin_amdgcn_raw_buffer_load_b16(src, off, 0, 0);
                hvals[q][0] = right ? b : (b << 16);
                hvals[q][1] = 0u;
            }
        } else {
            if constexpr (H == 1) {
                hvals[q][0] = __builtin_amdgcn_raw_buffer_load_b32(src, off, 0, 0);
            } else {
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(src, off, 0, 0);
                hvals[q][0] = v[0];
                hvals[q][1] = v[1];
            }
        }
    }
    // LDS writes are unconditional (idle lanes write a spare slot) so that
    // the loads above are not sunk into a branch.
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int it = (int)tid + q * NT;
        const int ry = it / G::CPR, c = it % G::CPR;
        const int slot = (NCHUNK % NT == 0 || it < NCHUNK) ? ry * G::PITCH + G::OFF + c * G::CB
                                                          : SPARE;
        *reinterpret_cast<LV *>(lds + slot) = vals[q];
    }
#pragma unroll
    for (int q = 0; q < NHIT; ++q) {
        const int it = (int)tid + q * NT;
        const bool ok = NHALO % NT == 0 || it < NHALO;
        const int rowb = (it >> 1) * G::PITCH;
        if constexpr (H == 1 || G::S == 1) {
            // one word: uint8 cells packed at its top (left) or bottom
            // (right) bytes, or one float32
            const int slot = ok ? rowb + 4 * ((it & 1) ? G::RIGHTW : G::OFFW - 1) : SPARE;
            *reinterpret_cast<uint32_t *>(lds + slot) = hvals[q][0];
        } else {
            const int slot = ok ? rowb + 4 * ((it & 1) ? G::RIGHTW : G::OFFW - 2) : SPARE;
            *reinterpret_cast<uint2 *>(lds + slot) = uint2{hvals[q][0], hvals[q][1]};
        }
    }
}

// New value of the output chunk at LDS row `rmd` (rows rmd-1 and rmd+1 above
// and below), chunk c, for global row y, masked to gasket members.
template <int RULE, int R>
__device__ __forceinline__ void chunk_update(const uint32_t *lw, int rmd, int c, uint32_t xc,
                                             uint32_t y, float alpha, float c1,
                                             uint32_t (&out)[Geom<RULE, R>::W])
{
    using G = Geom<RULE, R>;
    using V = typename VecT<G::CB>::T;
    const int base = G::OFFW + c * G::W;
    const int r_up = (rmd - 1) * G::PITCHW, r_md = rmd * G::PITCHW, r_dn = (rmd + 1) * G::PITCHW;
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

// Compute the tile's rows from an LDS buffer holding rows y0-1 .. y0+rho
// (layout as staged with H = 1) and store the chunks that hold a member.
template <int RULE, int R, int NT, int FL>
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
        chunk_update<RULE, R>(lw, j + 1, c, xc, y, alpha, c1, out);
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

// Value of one cell after a step, from a buffer staged with H = 2 (LDS row
// sr holds global row y, column offset dx from x0); 0 off the gasket.
template <int RULE, int R>
__device__ __forceinline__ uint32_t cell_update(const uint8_t *lds, int sr, int dx, uint32_t x,
                                                uint32_t y, float alpha, float c1)
{
    using G = Geom<RULE, R>;
    if ((x & y) != 0u)
        return 0u;
    auto at = [&](int row, int d) -> uint32_t {
        const uint8_t *q = lds + row * G::PITCH + G::OFF + d * G::S;
        if constexpr (G::S == 1)
            return *q;
        else
            return *reinterpret_cast<const uint32_t *>(q);
    };
    if constexpr (RULE == RULE_CA) {
        const uint32_t self = at(sr, dx);
        uint32_t cnt = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int ddx = -1; ddx <= 1; ++ddx)
                cnt += at(sr + dy, dx + ddx);
        cnt -= self; // the 8 neighbours
        return (cnt == 3u || (self == 1u && cnt == 2u)) ? 1u : 0u;
    } else {
        const float v = heat_cell(__uint_as_float(at(sr, dx)), __uint_as_float(at(sr - 1, dx)),
                                  __uint_as_float(at(sr + 1, dx)), __uint_as_float(at(sr, dx - 1)),
                                  __uint_as_float(at(sr, dx + 1)), alpha, c1);
        return __float_as_uint(v);
    }
}

// Intermediate step of the fused form: from the H = 2 staging (rows
// y0-2 .. y0+rho+1) compute rows y0-1 .. y0+rho and columns x0-1 .. x0+rho
// into the intermediate buffer, laid out as an H = 1 staging.
template <int RULE, int R, int NT>
__device__ __forceinline__ void mid_step(uint8_t *lds, const StepParams &p, uint32_t x0,
                                         uint32_t y0)
{
    using G = Geom<RULE, R>;
    using V = typename VecT<G::CB>::T;
    const uint32_t n = 1u << p.k;
    const uint32_t tid = threadIdx.x;
    const float alpha = p.alpha;
    const float c1 = 1.0f - 4.0f * alpha;
    const uint32_t *lw = reinterpret_cast<const uint32_t *>(lds);
    uint8_t *mid = lds + G::MID;
    constexpr int NMID = G::ROWS * G::CPR;
#pragma unroll
    for (int q = 0; q < (NMID + NT - 1) / NT; ++q) {
        const int it = (int)tid + q * NT;
        if (NMID % NT != 0 && it >= NMID)
            break;
        const int by = it / G::CPR, c = it % G::CPR; // intermediate row, chunk
        const int64_t yy = (int64_t)y0 - 1 + by;
        const uint32_t xc = x0 + (uint32_t)c * G::CCELLS;
        uint32_t out[G::W];
        if (yy < 0 || yy >= (int64_t)n || ((xc >> G::CLOG) & ((uint32_t)yy >> G::CLOG)) != 0u) {
#pragma unroll
            for (int w = 0; w < G::W; ++w)
                out[w] = 0u;
        } else {
            chunk_update<RULE, R>(lw, by + 1, c, xc, (uint32_t)yy, alpha, c1, out);
        }
        *reinterpret_cast<V *>(mid + by * G::PITCH + G::OFF + c * G::CB) = pack<G::W>(out);
    }
    // the one-cell ring's left and right columns
    for (int it = (int)tid; it < 2 * G::ROWS; it += NT) {
        const int by = it >> 1;
        const bool right = it & 1;
        const int64_t yy = (int64_t)y0 - 1 + by;
        const int64_t xx = right ? (int64_t)x0 + G::RHO : (int64_t)x0 - 1;
        uint32_t v = 0u;
        if (yy >= 0 && yy < (int64_t)n && xx >= 0 && xx < (int64_t)n)
            v = cell_update<RULE, R>(lds, by + 1, right ? G::RHO : -1, (uint32_t)xx,
                                     (uint32_t)yy, alpha, c1);
        uint32_t *wrow = reinterpret_cast<uint32_t *>(mid + by * G::PITCH);
        if constexpr (G::S == 1)
            wrow[right ? G::RIGHTW : G::OFFW - 1] = right ? v : (v << 24);
        else
            wrow[right ? G::RIGHTW : G::OFFW - 1] = v;
    }
}

// Process the tile whose top-left cell is (x0, y0): one step, or two with
// TILE_FUSE2.  All NT threads of the workgroup must call it (it contains
// workgroup barriers).
template <int RULE, int R, int NT, int FL = 0>
__device__ __forceinline__ void tile_step(uint8_t *lds, const StepParams &p,
                                          uint32_t x0, uint32_t y0)
{
    if constexpr ((FL & TILE_FUSE2) != 0 && Geom<RULE, R>::FUSABLE) {
        stage_tile<RULE, R, NT, FL, 2>(lds, p, x0, y0);
        __syncthreads();
        mid_step<RULE, R, NT>(lds, p, x0, y0);
        __syncthreads();
        store_tile<RULE, R, NT, FL>(lds + Geom<RULE, R>::MID, p, x0, y0);
    } else {
        stage_tile<RULE, R, NT, FL, 1>(lds, p, x0, y0);
        __syncthreads();
        store_tile<RULE, R, NT, FL>(lds, p, x0, y0);
    }
}

// LDS bytes a step kernel of this shape needs.
template <int RULE, int R, int FL>
constexpr int tile_lds_bytes()
{
    return ((FL & TILE_FUSE2) != 0 && Geom<RULE, R>::FUSABLE) ? Geom<RULE, R>::LDS2_BYTES
                                                              : Geom<RULE, R>::LDS_BYTES;
}

} // namespace fractal
