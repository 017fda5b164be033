// batch_kernels.hpp -- kernels of the batched step (one workgroup per tile,
// or persistent) and the table that picks an instantiation; each rule is
// instantiated in its own translation unit.
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

// Persistent form: workgroup b walks the contiguous tile ids
// [b*per, (b+1)*per) in order, so tiles that are neighbours in the gasket's
// self-similar order stay on one die and share its L2.
template <int RULE, int R, int NT, int FL>
__global__ __launch_bounds__(NT) void batch_persistent_kernel(
    const BatchEntry *__restrict__ table, int count, uint64_t total, int local_step)
{
    __shared__ __align__(16) uint8_t lds[tile_lds_bytes<RULE, R, FL>()];
    const uint64_t per = (total + gridDim.x - 1) / gridDim.x;
    const uint64_t w0 = (uint64_t)blockIdx.x * per;
    const uint64_t w1 = w0 + per < total ? w0 + per : total;
    if (w0 >= w1)
        return;
    int j = find_instance(table, count, w0);
    uint64_t next = j + 1 < count ? table[j + 1].tile_begin : ~0ull;
    for (uint64_t w = w0; w < w1; ++w) {
        while (w >= next) {
            ++j;
            next = j + 1 < count ? table[j + 1].tile_begin : ~0ull;
        }
        const BatchEntry e = table[j];
        __syncthreads(); // the previous tile's LDS reads are done
        batch_tile<RULE, R, NT, FL>(lds, e, (uint32_t)(w - e.tile_begin), local_step);
    }
}


template <int RULE, int NT, int FL>
static void pick_r(int r, TileFn *tf, PersistFn *pf)
{
    *tf = nullptr;
    *pf = nullptr;
    switch (r) {
#define FRACTAL_BATCH_CASE(RR)                                                                     \
    case RR:                                                                                       \
        if constexpr (!(fused_steps<FL>() > 1 && !Geom<RULE, RR>::FUSABLE) && !(NT == 256 && RR < 3)) { \
            *tf = batch_tile_kernel<RULE, RR, NT, FL>;                                             \
            *pf = batch_persistent_kernel<RULE, RR, NT, FL>;                                       \
        }                                                                                          \
        break;
        FRACTAL_BATCH_CASE(0)
        FRACTAL_BATCH_CASE(1)
        FRACTAL_BATCH_CASE(2)
        FRACTAL_BATCH_CASE(3)
        FRACTAL_BATCH_CASE(4)
        FRACTAL_BATCH_CASE(5)
        FRACTAL_BATCH_CASE(6)
        FRACTAL_BATCH_CASE(7)
#undef FRACTAL_BATCH_CASE
    default: break;
    }
}

template <int RULE, int FL>
static void pick_threads(int r, int threads, TileFn *tf, PersistFn *pf)
{
    if (threads == 256)
        pick_r<RULE, 256, FL>(r, tf, pf);
    else
        pick_r<RULE, 64, FL>(r, tf, pf);
}

template <int RULE>
static void pick_batch_kernel(int r, int threads, int flags, TileFn *tf, PersistFn *pf)
{
    switch (flags) {
    case 0: pick_threads<RULE, 0>(r, threads, tf, pf); break;
    case 1: pick_threads<RULE, 1>(r, threads, tf, pf); break;
    case 2: pick_threads<RULE, 2>(r, threads, tf, pf); break;
    case 3: pick_threads<RULE, 3>(r, threads, tf, pf); break;
    case 9: pick_threads<RULE, 9>(r, threads, tf, pf); break;
    case 11: pick_threads<RULE, 11>(r, threads, tf, pf); break;
    case 17: pick_threads<RULE, 17>(r, threads, tf, pf); break;
    case 19: pick_threads<RULE, 19>(r, threads, tf, pf); break;
    default:
        *tf = nullptr;
        *pf = nullptr;
    }
}

} // namespace fractal
