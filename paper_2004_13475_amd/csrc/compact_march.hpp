// compact_march.hpp -- the register-march step over compact storage.
//
// Compact layout (r fixed per state): the 3^(k-r) non-empty tiles of side
// rho = 2^r are stored in their curve order L (the order whose base-3 digits
// are the beta_mu, so lambda(L) is the tile's block), tile L's rho x rho box
// row-major at cell offset L * rho^2.  A lane finds the tiles around its own
// by lambda^-1 of their block coordinates, so the walk reads the same cell
// values as over the n x n array and the result is identical.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_map.hpp"
#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

// A lane's chunk column in compact storage: the tiles above, at and below its
// tile row (nullptr where there is no tile), within +-1 tile since T and the
// halo width are at most rho.
template <int R, int S>
struct CompactAddr {
    static constexpr int RHO = 1 << R;
    static constexpr int64_t ROWB = (int64_t)RHO * S; // bytes per tile row
    const uint8_t *up, *mid, *dn;
    const uint8_t *base; // the state's first tile: always readable
    uint8_t *dst;
    int y0; // first array row of the lane's tile row
    int n;
    __device__ __forceinline__ const uint8_t *col(int y) const
    {
        // one of three pointers by masks: a select between neighbouring
        // fields may otherwise become an indexed load from a stack copy
        const int s = (y - y0) >> R; // -1, 0 or 1
        const uint64_t mu = 0u - (uint64_t)(s < 0), md = 0u - (uint64_t)(s > 0);
        const uint64_t v = ((uint64_t)up & mu) | ((uint64_t)dn & md) |
                           ((uint64_t)mid & ~(mu | md));
        return reinterpret_cast<const uint8_t *>(v);
    }
    __device__ __forceinline__ bool has(int y) const
    {
        return (uint32_t)y < (uint32_t)n && col(y) != nullptr;
    }
    __device__ __forceinline__ const uint8_t *ld(int, int y) const
    {
        return col(y) + (int64_t)(y & (RHO - 1)) * ROWB;
    }
    __device__ __forceinline__ const uint8_t *any() const { return base; }
    __device__ __forceinline__ uint8_t *st(int, int y) const
    {
        return dst + (int64_t)(y & (RHO - 1)) * ROWB;
    }
};

struct CompactArgs {
    const uint8_t *src;
    uint8_t *dst;
    int k;
    float alpha;
    int rb;         // tile level k - r
    uint32_t total; // 3^rb tiles
    int band_log;
};
typedef void (*CompactFn)(CompactArgs);

template <int RULE, int R, int T, int HL>
constexpr bool compact_shape_ok()
{
    using M = MGeom<RULE, R, T, HL>;
    return M::VALID && march_supported(RULE, T, R) && T <= M::RHO && HL * M::CC <= M::RHO;
}

template <int RULE, int R, int T, int HL, int FL, int WPE, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void compact_march_kernel(CompactArgs a)
{
    using M = MGeom<RULE, R, T, HL>;
    static_assert(compact_shape_ok<RULE, R, T, HL>(), "compact march shape");
    const MarchLane<RULE, R, T, HL> ln;
    const uint32_t wg = xcd_chunk(blockIdx.x, gridDim.x);
    const uint32_t wave = wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t item = (uint64_t)wave * M::P + ln.grp; // (tile, band)
    const uint64_t tile = item >> a.band_log;
    const int band = (int)(item & ((1u << a.band_log) - 1u));
    const bool active = ln.grp < (uint32_t)M::P && tile < a.total;
    if (__builtin_amdgcn_ballot_w64(active) == 0u)
        return;
    TileXY t{0u, 0u};
    if (active)
        t = lambda_lane((uint32_t)tile, a.rb, FRACTAL_ORDER_CURVE);
    const int n = 1 << a.k;
    const int nb = 1 << a.rb;
    const int H = M::RHO >> a.band_log;
    const int xc = (int)(t.x << R) + ln.col * M::CC;
    const int ybase = (int)(t.y << R) + band * H;
    const int tx = xc >> R; // tile column of this lane's chunk (-1 left of the array)
    constexpr int64_t TB = (int64_t)M::RHO * M::RHO * M::S; // bytes per tile
    const int64_t coff = (int64_t)(xc & (M::RHO - 1)) * M::S;
    auto tile_col = [&](int dy) -> const uint8_t * {
        const int ty = (int)t.y + dy;
        const bool ex = active && tx >= 0 && tx < nb && ty >= 0 && ty < nb &&
                        ((tx & ty) == 0);
        return ex ? a.src + (int64_t)lambda_inverse((uint32_t)tx, (uint32_t)ty, a.rb) * TB + coff
                  : nullptr;
    };
    CompactAddr<R, M::S> A;
    A.up = tile_col(-1);
    A.mid = tile_col(0);
    A.dn = tile_col(1);
    A.base = a.src;
    A.dst = a.dst + (int64_t)tile * TB + coff; // used by the interior lanes only
    A.y0 = (int)(t.y << R);
    A.n = n;
    march_walk_at<RULE, R, T, HL, FL, D>(A, a.k, a.alpha, xc, ybase, H,
                                         active && xc >= 0 && xc < n,
                                         ln.col >= 0 && ln.col < M::IL);
}

template <int RULE, int R, int T, int FL>
static CompactFn compact_fn()
{
    constexpr int HL = march_hl(RULE, T);
    if constexpr (compact_shape_ok<RULE, R, T, HL>())
        return compact_march_kernel<RULE, R, T, HL, FL, march_wpe(T), march_depth(RULE, T)>;
    else
        return nullptr;
}

template <int RULE, int FL>
static CompactFn compact_pick_rt(int r, int T)
{
    switch (r) {
#define FRACTAL_COMPACT_R(RR)                                                                      \
    case RR:                                                                                       \
        switch (T) {                                                                               \
        case 1: return compact_fn<RULE, RR, 1, FL>();                                              \
        case 2: return compact_fn<RULE, RR, 2, FL>();                                              \
        case 4: return compact_fn<RULE, RR, 4, FL>();                                              \
        case 8: return compact_fn<RULE, RR, 8, FL>();                                              \
        case 16: return compact_fn<RULE, RR, 16, FL>();                                            \
        default: return nullptr;                                                                   \
        }
        FRACTAL_COMPACT_R(2)
        FRACTAL_COMPACT_R(3)
        FRACTAL_COMPACT_R(4)
        FRACTAL_COMPACT_R(5)
        FRACTAL_COMPACT_R(6)
        FRACTAL_COMPACT_R(7)
#undef FRACTAL_COMPACT_R
    default: return nullptr;
    }
}

CompactFn pick_compact_ca(int r, int T, bool nt);
CompactFn pick_compact_heat(int r, int T, bool nt);

} // namespace fractal
