// batch_kernels.hpp -- the LDS-engine kernel of the batched step (one
// workgroup per tile) and the table that picks an instantiation; each rule
// is instantiated in its own translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "device_tile.hpp"
#include "internal.hpp"

namespace fractal {

// Last of entries [0, count) whose range starts at or before w (entries are
// sorted by tile_begin).
__device__ __forceinline__ int find_instance(const BatchEntry *__restrict__ table, int count,
                                             uint64_t w)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].tile_begin <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// `slot` is the index of this launch within the item's launches of this
// list's size; every launch flips the buffers.
template <int RULE, int R, int NT, int FL>
__device__ __forceinline__ void batch_tile(uint8_t *lds, const BatchEntry &e, uint32_t L,
                                           int slot)
{
    const TileXY t = lambda_wave_curve(L, e.k - R);
    const int flips = e.flip0 + slot;
    const bool odd = ((e.phase + flips) & 1) != 0;
    StepParams p;
    p.src = odd ? e.buf1 : e.buf0;
    p.dst = odd ? e.buf0 : e.buf1;
    p.k = e.k;
    p.alpha = e.alpha;
    tile_step<RULE, R, NT, FL>(lds, p, t.x << R, t.y << R);
}

// One workgroup per tile of the class's work list, ids laid out per die in
// contiguous ranges as in the lambda step kernels.  The grid is 2-D only to
// stay inside launch limits; workgroups past the end return at once.
template <int RULE, int R, int NT, int FL>
__global__ __launch_bounds__(NT) void batch_tile_kernel(const BatchEntry *__restrict__ table,
                                                        int count, uint32_t total,
                                                        int local_step)
{
    __shared__ __align__(16) uint8_t lds[tile_lds_bytes<RULE, R, FL>()];
    const uint32_t lin = blockIdx.y * gridDim.x + blockIdx.x;
    if (lin >= total)
        return;
    const uint32_t w = xcd_chunk(lin, total);
    const BatchEntry e = table[find_instance(table, count, w)];
    batch_tile<RULE, R, NT, FL>(lds, e, (uint32_t)(w - e.tile_begin), local_step);
}

template <int RULE, int NT, int FL>
static TileFn pick_r(int r)
{
    switch (r) {
#define FRACTAL_BATCH_CASE(RR)                                                                     \
    case RR:                                                                                       \
        if constexpr (!(fused_steps<FL>() > 1 && !Geom<RULE, RR>::FUSABLE) && !(NT == 256 && RR < 3)) \
            return batch_tile_kernel<RULE, RR, NT, FL>;                                            \
        return nullptr;
        FRACTAL_BATCH_CASE(0)
        FRACTAL_BATCH_CASE(1)
        FRACTAL_BATCH_CASE(2)
        FRACTAL_BATCH_CASE(3)
        FRACTAL_BATCH_CASE(4)
        FRACTAL_BATCH_CASE(5)
        FRACTAL_BATCH_CASE(6)
        FRACTAL_BATCH_CASE(7)
#undef FRACTAL_BATCH_CASE
    default: return nullptr;
    }
}

template <int RULE, int FL>
static TileFn pick_threads(int r, int threads)
{
    return threads == 256 ? pick_r<RULE, 256, FL>(r) : pick_r<RULE, 64, FL>(r);
}

template <int RULE>
static TileFn pick_batch_kernel(int r, int threads, int flags)
{
    switch (flags) {
    case 0: return pick_threads<RULE, 0>(r, threads);
    case 1: return pick_threads<RULE, 1>(r, threads);
    case 2: return pick_threads<RULE, 2>(r, threads);
    case 3: return pick_threads<RULE, 3>(r, threads);
    case 9: return pick_threads<RULE, 9>(r, threads);
    case 11: return pick_threads<RULE, 11>(r, threads);
    case 17: return pick_threads<RULE, 17>(r, threads);
    case 19: return pick_threads<RULE, 19>(r, threads);
    default: return nullptr;
    }
}

} // namespace fractal
