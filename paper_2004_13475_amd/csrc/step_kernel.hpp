// step_kernel.hpp -- the lambda / bounding-box / matrix-core step kernel
// template and the table that picks an instantiation at run time.  Each map
// is instantiated in its own translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "device_tile.hpp"
#include "internal.hpp"

namespace fractal {

// One workgroup per tile.  lambda maps: the grid is the compact 3^ceil(rb/2)
// x 3^floor(rb/2) orthotope.  Bounding box: the grid is n_b x n_b and a
// workgroup on an empty tile returns before touching memory.
template <int RULE, int R, int NT, int MAP, int FL>
__global__ __launch_bounds__(NT) void step_kernel(StepLaunchArgs a)
{
    __shared__ __align__(16) uint8_t lds[tile_lds_bytes<RULE, R, FL>()];
    const uint32_t lin = blockIdx.y * gridDim.x + blockIdx.x;
    TileXY t;
    if constexpr (MAP == MAP_BB) {
        const uint32_t id = a.order != FRACTAL_ORDER_NATURAL ? xcd_chunk(lin, a.total) : lin;
        t.x = id & ((1u << a.rb) - 1u);
        t.y = id >> a.rb;
        if ((t.x & t.y) != 0u)
            return; // empty block: nothing of the gasket here
    } else if (a.order == FRACTAL_ORDER_NATURAL) {
        const uint32_t wx = blockIdx.x, wy = blockIdx.y;
        if constexpr (MAP == MAP_MFMA)
            t = lambda_mfma([&](uint32_t mu) { return beta_of_omega(wx, wy, mu); }, a.rb);
        else
            t = lambda_wave(wx, wy, a.rb);
    } else {
        const uint32_t L = a.order == FRACTAL_ORDER_CURVE_XCD ? xcd_chunk(lin, a.total) : lin;
        if constexpr (MAP == MAP_MFMA)
            t = lambda_mfma(
                [&](uint32_t mu) {
                    const uint32_t q = L / pow3_u32(mu - 1u);
                    return q - 3u * (q / 3u);
                },
                a.rb);
        else
            t = lambda_wave_curve(L, a.rb);
    }
    StepParams p;
    p.src = a.src;
    p.dst = a.dst;
    p.k = a.k;
    p.alpha = a.alpha;
    tile_step<RULE, R, NT, FL>(lds, p, t.x << R, t.y << R);
}

template <int MAP, int RULE, int NT, int FL>
static StepFn pick_r(int r)
{
    // two-step fusion exists only for tiles with rows of >= 16 bytes
    switch (r) {
#define FRACTAL_STEP_CASE(RR)                                                                      \
    case RR:                                                                                       \
        if constexpr (fused_steps<FL>() > 1 && !Geom<RULE, RR>::FUSABLE)                           \
            return nullptr;                                                                        \
        else if constexpr (NT == 256 && RR < 3)                                                    \
            return nullptr;                                                                        \
        else                                                                                       \
            return step_kernel<RULE, RR, NT, MAP, FL>;
        FRACTAL_STEP_CASE(0)
        FRACTAL_STEP_CASE(1)
        FRACTAL_STEP_CASE(2)
        FRACTAL_STEP_CASE(3)
        FRACTAL_STEP_CASE(4)
        FRACTAL_STEP_CASE(5)
        FRACTAL_STEP_CASE(6)
        FRACTAL_STEP_CASE(7)
#undef FRACTAL_STEP_CASE
    default: return nullptr;
    }
}

template <int MAP, int RULE, int FL>
static StepFn pick_threads(int r, int threads)
{
    return threads == 256 ? pick_r<MAP, RULE, 256, FL>(r) : pick_r<MAP, RULE, 64, FL>(r);
}

template <int MAP, int FL>
static StepFn pick_rule(int rule, int r, int threads)
{
    return rule == FRACTAL_RULE_CA ? pick_threads<MAP, RULE_CA, FL>(r, threads)
                                   : pick_threads<MAP, RULE_HEAT, FL>(r, threads);
}

template <int MAP>
static StepFn pick_step_kernel(int rule, int r, int threads, int flags)
{
    switch (flags) {
    case 0: return pick_rule<MAP, 0>(rule, r, threads);
    case 1: return pick_rule<MAP, 1>(rule, r, threads);
    case 2: return pick_rule<MAP, 2>(rule, r, threads);
    case 3: return pick_rule<MAP, 3>(rule, r, threads);
    case 9: return pick_rule<MAP, 9>(rule, r, threads);
    case 11: return pick_rule<MAP, 11>(rule, r, threads);
    case 17: return pick_rule<MAP, 17>(rule, r, threads);
    case 19: return pick_rule<MAP, 19>(rule, r, threads);
    default: return nullptr;
    }
}

} // namespace fractal
