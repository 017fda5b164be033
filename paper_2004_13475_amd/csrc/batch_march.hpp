// batch_march.hpp -- the register-march engine over a batch work list:
// each lane group finds its instance by the tile prefix, then walks that
// instance's tile as the single-gasket march kernel does.  Instantiated per
// rule in batch_march_ca.hip and batch_march_heat.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "batch_kernels.hpp"
#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

// Items (tile, band) of the list in order, P per wavefront and four
// wavefronts per workgroup item; tile id w of the list is local tile
// w - tile_begin of its instance, taken along the gasket's self-similar
// order.  `slot` is the index of this launch within the list (the entry's
// flip0 + slot launches precede it).  The `groups` workgroup items are split
// into 8 contiguous ranges, one per accelerator die (hardware workgroup b
// runs on die b % 8); the workgroups of a die stride through its range.  A
// grid of `groups` workgroups takes one item each (the die-contiguous order
// of the lambda step kernels); a persistent grid of fewer workgroups, as
// many as the chip holds at once, walks several items each.
template <int RULE, int R, int T, int HL, int FL, int WPE, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void batch_march_kernel(const BatchEntry *__restrict__ table, int count, uint64_t total,
                        int band_log, int slot, uint32_t groups)
{
    using M = MGeom<RULE, R, T, HL>;
    static_assert(M::VALID, "march shape");
    const MarchLane<RULE, R, T, HL> ln;
    const uint32_t die = blockIdx.x & 7u, q = blockIdx.x >> 3;
    const uint32_t per = groups >> 3, rem = groups & 7u;
    const uint32_t lo = die * per + (die < rem ? die : rem);
    const uint32_t hi = lo + per + (die < rem ? 1u : 0u);
    const uint32_t stride = (gridDim.x >> 3) + (die < (gridDim.x & 7u) ? 1u : 0u);
    // Idle lanes still issue the walk's loads, from a readable chunk: the
    // first instance's state (the list is not empty).
    const uint8_t *any = table[0].buf0;
    for (uint32_t g = lo + q; g < hi; g += stride) {
        const uint32_t wave = g * (blockDim.x >> 6) + (threadIdx.x >> 6);
        const uint64_t item = (uint64_t)wave * M::P + ln.grp;
        const uint64_t w = item >> band_log;
        const int band = (int)(item & ((1u << band_log) - 1u));
        const bool active = ln.grp < (uint32_t)M::P && w < total;
        if (__builtin_amdgcn_ballot_w64(active) == 0u)
            continue; // wavefront-uniform
        const uint8_t *src = any;
        uint8_t *dst = nullptr;
        int k = R;
        float alpha = 0.0f;
        TileXY t{0u, 0u};
        if (active) {
            const BatchEntry e = table[find_instance(table, count, w)];
            t = lambda_lane((uint32_t)(w - e.tile_begin), e.k - R, FRACTAL_ORDER_CURVE);
            const bool odd = ((e.phase + e.flip0 + slot) & 1) != 0;
            src = odd ? e.buf1 : e.buf0;
            dst = odd ? e.buf0 : e.buf1;
            k = e.k;
            alpha = e.alpha;
        }
        march_walk<RULE, R, T, HL, FL, D>(src, dst, k, alpha, t, band, band_log, active, ln.col);
    }
}

template <int RULE, int R, int T, int FL>
static BatchMarchFn bm_fn()
{
    constexpr int HL = march_hl(RULE, T);
    if constexpr (MGeom<RULE, R, T, HL>::VALID && march_supported(RULE, T, R))
        return batch_march_kernel<RULE, R, T, HL, FL, march_wpe(T), march_depth(RULE, T)>;
    else
        return nullptr;
}

template <int RULE, int FL>
static BatchMarchFn bm_pick(int r, int T)
{
    switch (r) {
#define FRACTAL_BM_R(RR)                                                                           \
    case RR:                                                                                       \
        switch (T) {                                                                               \
        case 1: return bm_fn<RULE, RR, 1, FL>();                                                   \
        case 2: return bm_fn<RULE, RR, 2, FL>();                                                   \
        case 4: return bm_fn<RULE, RR, 4, FL>();                                                   \
        case 8: return bm_fn<RULE, RR, 8, FL>();                                                   \
        case 16: return bm_fn<RULE, RR, 16, FL>();                                                   \
        default: return nullptr;                                                                   \
        }
        FRACTAL_BM_R(2)
        FRACTAL_BM_R(3)
        FRACTAL_BM_R(4)
        FRACTAL_BM_R(5)
        FRACTAL_BM_R(6)
        FRACTAL_BM_R(7)
#undef FRACTAL_BM_R
    default: return nullptr;
    }
}

template <int RULE>
static BatchMarchFn bm_pick_rule(int r, int T, bool nt)
{
    return nt ? bm_pick<RULE, TILE_NT_STORE>(r, T) : bm_pick<RULE, 0>(r, T);
}

} // namespace fractal
