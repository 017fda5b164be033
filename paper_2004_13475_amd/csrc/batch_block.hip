// batch_block.hip -- the block engines over a batch work list: instances
// on 64 x 64 tiles, one wavefront per tile of the list.
#include <hip/hip_runtime.h>

#include "batch_kernels.hpp"
#include "block_ca.hpp"
#include "block_heat.hpp"
#include "internal.hpp"

namespace fractal {

// Wavefront w of the grid takes tile id w of the list: its instance from the
// per-instance tile prefix, its tile from that instance's lambda in the
// curve order (per wavefront).  `slot` is the index of this launch within
// the item's launches of this list's size (every launch flips the buffers);
// every launch of the list advances `steps` steps (at most D: the class's
// halo, 16 or 32 cells).
template <int FL, int D>
__global__ __launch_bounds__(256) void batch_block_heat_kernel(const BatchEntry *__restrict__ table,
                                                               int count, uint64_t total,
                                                               int slot, int steps)
{
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= total)
        return; // wavefront-uniform
    const BatchEntry e = table[find_instance(table, count, w)];
    const TileXY t = lambda_wave_curve((uint32_t)(w - e.tile_begin), e.k - blk::kTileLog);
    const bool odd = ((e.phase + e.flip0 + slot) & 1) != 0;
    block_tile<FL, D>(odd ? e.buf1 : e.buf0, odd ? e.buf0 : e.buf1, e.k, e.alpha, t, steps);
}

template <int FL, int D>
__global__ __launch_bounds__(256) void batch_block_ca_kernel(const BatchEntry *__restrict__ table,
                                                             int count, uint64_t total, int slot,
                                                             int steps)
{
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= total)
        return; // wavefront-uniform
    const BatchEntry e = table[find_instance(table, count, w)];
    const TileXY t = lambda_wave_curve((uint32_t)(w - e.tile_begin), e.k - blk::kTileLog);
    const bool odd = ((e.phase + e.flip0 + slot) & 1) != 0;
    block_ca_tile<FL, D>(odd ? e.buf1 : e.buf0, odd ? e.buf0 : e.buf1, e.k, t, steps);
}

template <int D>
static BatchBlockFn pick_batch_block_d(int rule, bool nt)
{
    if (rule == FRACTAL_RULE_CA)
        return nt ? batch_block_ca_kernel<TILE_NT_STORE, D> : batch_block_ca_kernel<0, D>;
    return nt ? batch_block_heat_kernel<TILE_NT_STORE, D> : batch_block_heat_kernel<0, D>;
}

BatchBlockFn pick_batch_block(int rule, bool nt, int depth)
{
    return depth == 16 ? pick_batch_block_d<16>(rule, nt)
           : depth == 32 ? pick_batch_block_d<32>(rule, nt)
                         : nullptr;
}

} // namespace fractal
