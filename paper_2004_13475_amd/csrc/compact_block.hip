// compact_block.hip -- the block engines over compact storage of 64 x 64
// tiles: one wavefront per tile in curve order (tile L of the state is
// lambda's tile L), the tile and the neighbours a launch reads found by
// their curve indices (lambda^-1), so the steps read the same cell values as
// over the n x n array and give the same bits.
#include <hip/hip_runtime.h>

#include "block_ca.hpp"
#include "block_heat.hpp"
#include "internal.hpp"

namespace fractal {

template <int RULE, int FL, int D>
__global__ __launch_bounds__(256) void compact_block_kernel(BlockArgs a)
{
    uint32_t wg = blockIdx.x;
    if (a.order == FRACTAL_ORDER_CURVE_XCD)
        wg = xcd_chunk(wg, gridDim.x);
    const uint32_t L = wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (L >= a.total)
        return; // wavefront-uniform
    const TileXY t = lambda_wave_curve(L, a.rb);
    const blk::CompactLayout lay = blk::compact_layout(t, L, a.rb, RULE == RULE_CA ? 1 : 4);
    if constexpr (RULE == RULE_CA)
        block_ca_tile<FL, D>(a.src, a.dst, a.k, t, a.steps, lay);
    else
        block_tile<FL, D>(a.src, a.dst, a.k, a.alpha, t, a.steps, lay);
}

template <int RULE, int D>
static BlockFn pick_compact_block_d(bool nt)
{
    return nt ? compact_block_kernel<RULE, TILE_NT_STORE, D> : compact_block_kernel<RULE, 0, D>;
}

static BlockFn pick_compact_block(int rule, bool nt, int depth)
{
    const bool ca = rule == FRACTAL_RULE_CA;
    switch (depth) {
    case 16:
        return ca ? pick_compact_block_d<RULE_CA, 16>(nt) : pick_compact_block_d<RULE_HEAT, 16>(nt);
    case 24:
        return ca ? pick_compact_block_d<RULE_CA, 24>(nt) : pick_compact_block_d<RULE_HEAT, 24>(nt);
    case 32:
        return ca ? pick_compact_block_d<RULE_CA, 32>(nt) : pick_compact_block_d<RULE_HEAT, 32>(nt);
    case 36:
        return ca ? pick_compact_block_d<RULE_CA, 36>(nt) : pick_compact_block_d<RULE_HEAT, 36>(nt);
    default:
        return nullptr;
    }
}

// Launches as for the n x n array: the fewest whose count has the parity of
// `steps` (the result lands in buf[steps & 1]), each of at most `cap` steps,
// the steps shared out evenly.
int launch_compact_block(int k, int rule, float alpha, void *c0, void *c1, int steps, int cap,
                         bool nt, hipStream_t s)
{
    if (k < blk::kTileLog || k - blk::kTileLog > 16)
        return set_error(FRACTAL_E_INVAL, "compact block launches need 6 <= k <= 22 (k = %d)", k);
    const int depth = cap <= 16 ? 16 : (cap <= 24 ? 24 : (cap <= 32 ? 32 : 36));
    BlockFn fn = pick_compact_block(rule, nt, depth);
    if (!fn || cap < 1 || cap > 36)
        return set_error(FRACTAL_E_INVAL, "no compact block kernel for %d steps per launch", cap);
    if (steps <= 0)
        return FRACTAL_OK;
    int L = (steps + cap - 1) / cap;
    if ((L & 1) != (steps & 1))
        ++L;
    BlockArgs a;
    a.k = k;
    a.alpha = alpha;
    a.rb = k - blk::kTileLog;
    a.order = FRACTAL_ORDER_CURVE;
    a.total = (uint32_t)pow3_u64(a.rb);
    uint8_t *bufs[2] = {static_cast<uint8_t *>(c0), static_cast<uint8_t *>(c1)};
    const uint64_t grid = ((uint64_t)a.total + 3u) / 4u;
    for (int i = 0; i < L; ++i) {
        a.steps = steps / L + (i < steps % L ? 1 : 0);
        a.src = bufs[i & 1];
        a.dst = bufs[(i + 1) & 1];
        void *args[] = {&a};
        hipError_t e = hipLaunchKernel((const void *)fn, dim3((unsigned)grid), dim3(256), args, 0, s);
        if (e != hipSuccess)
            return hip_error(e, "compact block launch");
    }
    return hip_error(hipGetLastError(), "compact block launch");
}

} // namespace fractal
