// block_heat.hip -- the block engine of the float32 heat step on one
// gasket (lambda and bounding-box maps), and the launcher of both block
// engines (the automaton's kernels are in block_ca.hip).
#include <hip/hip_runtime.h>

#include "block_heat.hpp"
#include "internal.hpp"

namespace fractal {

// One wavefront per tile: tile id `wave` of the map (lambda: the curve or
// natural order; BB: row-major over all (n/64)^2 tiles, empty ones idle).
template <int MAP, int FL, int D>
__global__ __launch_bounds__(256) void block_heat_kernel(BlockArgs a)
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
    block_tile<FL, D>(a.src, a.dst, a.k, a.alpha, t, a.steps);
}

// The two-slot form: one wavefront per 128 x 128 tile, up to 36 steps.
template <int MAP, int FL>
__global__ __launch_bounds__(256) void block2_heat_kernel(BlockArgs a)
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
    block2_tile<FL>(a.src, a.dst, a.k, a.alpha, t, a.steps, blk::ArrayLayout{(int64_t)4 << a.k, 4, t});
}

static BlockFn pick_block2(int map, bool nt)
{
    if (map == MAP_BB)
        return nt ? block2_heat_kernel<MAP_BB, TILE_NT_STORE> : block2_heat_kernel<MAP_BB, 0>;
    if (map == MAP_LAMBDA)
        return nt ? block2_heat_kernel<MAP_LAMBDA, TILE_NT_STORE> : block2_heat_kernel<MAP_LAMBDA, 0>;
    return nullptr;
}

template <int MAP, int D>
static BlockFn pick_block_d(bool nt)
{
    return nt ? block_heat_kernel<MAP, TILE_NT_STORE, D> : block_heat_kernel<MAP, 0, D>;
}

// The heat kernel for launches of up to `depth` steps (16, 24, 32 or 36).
static BlockFn pick_block(int map, bool nt, int depth)
{
    if (map != MAP_BB && map != MAP_LAMBDA)
        return nullptr;
    const bool bb = map == MAP_BB;
    switch (depth) {
    case 16:
        return bb ? pick_block_d<MAP_BB, 16>(nt) : pick_block_d<MAP_LAMBDA, 16>(nt);
    case 24:
        return bb ? pick_block_d<MAP_BB, 24>(nt) : pick_block_d<MAP_LAMBDA, 24>(nt);
    case 32:
        return bb ? pick_block_d<MAP_BB, 32>(nt) : pick_block_d<MAP_LAMBDA, 32>(nt);
    case 36:
        return bb ? pick_block_d<MAP_BB, 36>(nt) : pick_block_d<MAP_LAMBDA, 36>(nt);
    default:
        return nullptr;
    }
}

// Launches: the fewest whose count has the parity of `steps` (the result
// lands in buf[steps & 1]), each of at most the tuning's steps per launch,
// the steps shared out evenly (the kernel takes its step count at launch).
int launch_block(int map, int k, int rule, float alpha, void *b0, void *b1, int steps,
                 const fractal_tuning &t, hipStream_t s)
{
    // 64 x 64 tiles (one block per lane) or 128 x 128 tiles (two)
    const bool two = t.r == blk::kTile2Log;
    if ((t.r != blk::kTileLog && !two) || k < t.r)
        return set_error(FRACTAL_E_INVAL, "the block engine runs on 64 x 64 or 128 x 128 tiles "
                                          "(r = 6 or 7)");
    const int cap = launch_steps_of(t.flags);
    const bool nt = (t.flags & FRACTAL_FLAG_NT_STORE) != 0;
    // the kernel whose halo covers `cap` steps: 16 cells up to 16 steps,
    // then 24, 32 and 36 (the two-slot form: 36)
    const int depth = cap <= 16 ? 16 : (cap <= 24 ? 24 : (cap <= 32 ? 32 : 36));
    BlockFn fn = two ? (rule == FRACTAL_RULE_CA ? pick_block2_ca(map, nt) : pick_block2(map, nt))
                 : rule == FRACTAL_RULE_CA ? pick_block_ca(map, nt, depth)
                                           : pick_block(map, nt, depth);
    if (!fn || cap < 1 || cap > 36)
        return set_error(FRACTAL_E_INVAL, "no block kernel for map %d, rule %d, %d steps per launch",
                         map, rule, cap);
    if (steps <= 0)
        return FRACTAL_OK;
    int L = (steps + cap - 1) / cap;
    if ((L & 1) != (steps & 1))
        ++L;
    const int rb = k - t.r;
    BlockArgs a;
    a.k = k;
    a.alpha = alpha;
    a.rb = rb;
    a.order = t.order;
    a.total = map == MAP_BB ? (uint32_t)1u << (2 * rb) : (uint32_t)pow3_u64(rb);
    uint8_t *bufs[2] = {static_cast<uint8_t *>(b0), static_cast<uint8_t *>(b1)};
    const uint64_t grid = ((uint64_t)a.total + 3u) / 4u;
    for (int i = 0; i < L; ++i) {
        a.steps = steps / L + (i < steps % L ? 1 : 0);
        a.src = bufs[i & 1];
        a.dst = bufs[(i + 1) & 1];
        void *args[] = {&a};
        hipError_t e = hipLaunchKernel((const void *)fn, dim3((unsigned)grid), dim3(256), args, 0, s);
        if (e != hipSuccess)
            return hip_error(e, "block kernel launch");
    }
    return hip_error(hipGetLastError(), "block kernel launch");
}

} // namespace fractal
