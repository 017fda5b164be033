// block_ca.hip -- the block engine of the automaton on one gasket (lambda
// and bounding-box maps).
#include <hip/hip_runtime.h>

#include "block_ca.hpp"
#include "internal.hpp"

namespace fractal {

// One wavefront per tile: tile id `tile` of the map (lambda: the curve or
// natural order; BB: row-major over all (n/64)^2 tiles, empty ones idle).
template <int MAP, int FL, int D>
__global__ __launch_bounds__(256) void block_ca_kernel(BlockArgs a)
{
    uint32_t wg = blockIdx.x;
    if (a.order == FRACTAL_ORDER_CURVE_XCD)
        wg = xcd_chunk(wg, gridDim.x);
    const uint32_t tile = wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= a.total)
        return; // wavefront-uniform
    TileXY t;
    if constexpr (MAP == MAP_BB) {
        t.x = tile & ((1u << a.rb) - 1u);
        t.y = tile >> a.rb;
        if (t.x & t.y)
            return; // empty tile: the whole wavefront leaves
    } else if (a.order == FRACTAL_ORDER_NATURAL) {
        const uint32_t gx = pow3_u32((uint32_t)(a.rb + 1) / 2u);
        t = lambda_wave(tile % gx, tile / gx, a.rb);
    } else {
        t = lambda_wave_curve(tile, a.rb);
    }
    block_ca_tile<FL, D>(a.src, a.dst, a.k, t, a.steps);
}

// The two-slot form: one wavefront per 128 x 128 tile, up to 36 steps.
template <int MAP, int FL>
__global__ __launch_bounds__(256) void block2_ca_kernel(BlockArgs a)
{
    uint32_t wg = blockIdx.x;
    if (a.order == FRACTAL_ORDER_CURVE_XCD)
        wg = xcd_chunk(wg, gridDim.x);
    const uint32_t tile = wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= a.total)
        return; // wavefront-uniform
    TileXY t;
    if constexpr (MAP == MAP_BB) {
        t.x = tile & ((1u << a.rb) - 1u);
        t.y = tile >> a.rb;
        if (t.x & t.y)
            return; // empty tile: the whole wavefront leaves
    } else if (a.order == FRACTAL_ORDER_NATURAL) {
        const uint32_t gx = pow3_u32((uint32_t)(a.rb + 1) / 2u);
        t = lambda_wave(tile % gx, tile / gx, a.rb);
    } else {
        t = lambda_wave_curve(tile, a.rb);
    }
    block2_ca_tile<FL>(a.src, a.dst, a.k, t, a.steps,
                       blk::ArrayLayout{(int64_t)1 << a.k, 1, t, blk::kTile2Log});
}

BlockFn pick_block2_ca(int map, bool nt)
{
    if (map == MAP_BB)
        return nt ? block2_ca_kernel<MAP_BB, TILE_NT_STORE> : block2_ca_kernel<MAP_BB, 0>;
    if (map == MAP_LAMBDA)
        return nt ? block2_ca_kernel<MAP_LAMBDA, TILE_NT_STORE> : block2_ca_kernel<MAP_LAMBDA, 0>;
    return nullptr;
}

template <int MAP, int D>
static BlockFn pick_block_ca_d(bool nt)
{
    return nt ? block_ca_kernel<MAP, TILE_NT_STORE, D> : block_ca_kernel<MAP, 0, D>;
}

BlockFn pick_block_ca(int map, bool nt, int depth)
{
    if (map != MAP_BB && map != MAP_LAMBDA)
        return nullptr;
    const bool bb = map == MAP_BB;
    switch (depth) {
    case 16:
        return bb ? pick_block_ca_d<MAP_BB, 16>(nt) : pick_block_ca_d<MAP_LAMBDA, 16>(nt);
    case 24:
        return bb ? pick_block_ca_d<MAP_BB, 24>(nt) : pick_block_ca_d<MAP_LAMBDA, 24>(nt);
    case 32:
        return bb ? pick_block_ca_d<MAP_BB, 32>(nt) : pick_block_ca_d<MAP_LAMBDA, 32>(nt);
    case 36:
        return bb ? pick_block_ca_d<MAP_BB, 36>(nt) : pick_block_ca_d<MAP_LAMBDA, 36>(nt);
    default:
        return nullptr;
    }
}

} // namespace fractal
