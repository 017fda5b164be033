// step_kernels.hip -- lambda(omega) map kernels and the host launcher of the
// lambda / bounding-box / matrix-core step kernels.
#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "internal.hpp"

namespace fractal {

// ------------------------------------------------------------------ map
// Four wavefronts per workgroup; wavefront w of workgroup b evaluates omega
// number 4*b + w (row-major over the compact grid), then every further
// 4*gridDim.x-th.  Lane 0 writes the pair.
template <bool MFMA>
__global__ __launch_bounds__(256) void lambda_map_kernel(uint32_t *xy, int rb,
                                                         uint32_t gx,
                                                         uint64_t total)
{
    const uint64_t wave = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint64_t stride = (uint64_t)gridDim.x * 4u;
    for (uint64_t i = wave; i < total; i += stride) {
        const uint32_t wx = (uint32_t)(i % gx), wy = (uint32_t)(i / gx);
        TileXY t;
        if constexpr (MFMA)
            t = lambda_mfma([&](uint32_t mu) { return beta_of_omega(wx, wy, mu); }, rb);
        else
            t = lambda_wave(wx, wy, rb);
        if ((threadIdx.x & 63u) == 0u) {
            xy[2 * i + 0] = t.x;
            xy[2 * i + 1] = t.y;
        }
    }
}

int launch_lambda_map(int k, int r, uint32_t *d_xy, bool mfma, hipStream_t s)
{
    const int rb = k - r;
    const uint64_t gx = pow3_u64((rb + 1) / 2), gy = pow3_u64(rb / 2);
    const uint64_t total = gx * gy;
    const uint64_t want = (total + 3) / 4;
    const unsigned grid = (unsigned)(want < (1u << 20) ? want : (1u << 20));
    if (mfma)
        hipLaunchKernelGGL(lambda_map_kernel<true>, dim3(grid), dim3(256), 0, s,
                           d_xy, rb, (uint32_t)gx, total);
    else
        hipLaunchKernelGGL(lambda_map_kernel<false>, dim3(grid), dim3(256), 0, s,
                           d_xy, rb, (uint32_t)gx, total);
    return hip_error(hipGetLastError(), "lambda map launch");
}

// The per-lane form of the map (lambda_lane, as the register-march kernels
// evaluate it): thread i writes the block of tile id i in dispatch order
// `order`.
__global__ __launch_bounds__(256) void lambda_tiles_kernel(uint32_t *xy, int rb, int order,
                                                           uint32_t total)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const TileXY t = lambda_lane(i, rb, order);
        xy[2 * (uint64_t)i + 0] = t.x;
        xy[2 * (uint64_t)i + 1] = t.y;
    }
}

int launch_lambda_tiles(int rb, int order, uint32_t *d_xy, hipStream_t s)
{
    const uint64_t total = pow3_u64(rb);
    const uint64_t want = (total + 255) / 256;
    const unsigned grid = (unsigned)(want < (1u << 20) ? want : (1u << 20));
    hipLaunchKernelGGL(lambda_tiles_kernel, dim3(grid), dim3(256), 0, s, d_xy, rb, order,
                       (uint32_t)total);
    return hip_error(hipGetLastError(), "lambda tiles launch");
}

int launch_steps(int map, int k, int rule, float alpha, void *b0, void *b1,
                 int steps, const fractal_tuning &t, hipStream_t s)
{
    // T-step launches come in pairs so that the result still lands in
    // buf[steps & 1]; the remaining 0..2T-1 steps run one step per launch.
    if (t.flags & FRACTAL_FLAG_MARCH)
        return launch_march(map, k, rule, alpha, b0, b1, steps, t, s);
    if (t.flags & FRACTAL_FLAG_BLOCK)
        return launch_block(map, k, rule, alpha, b0, b1, steps, t, s);
    const int T = launch_steps_of(t.flags);
    const bool fuse = T > 1;
    const int fused = fuse ? 2 * (steps / (2 * T)) : 0;
    StepFn fn1 = pick_step(map, rule, t.r, t.threads,
                           t.flags & ~kFuseFlags);
    StepFn fn2 = fuse ? pick_step(map, rule, t.r, t.threads, t.flags) : nullptr;
    if (!fn1 || (fuse && !fn2))
        return set_error(FRACTAL_E_INVAL, "no kernel for map %d rule %d r %d threads %d flags %d",
                         map, rule, t.r, t.threads, t.flags);
    const int rb = k - t.r;
    dim3 grid;
    if (map == MAP_BB)
        grid = dim3(1u << rb, 1u << rb);
    else
        grid = dim3((unsigned)pow3_u64((rb + 1) / 2), (unsigned)pow3_u64(rb / 2));
    StepLaunchArgs a;
    a.k = k;
    a.alpha = alpha;
    a.rb = rb;
    a.order = t.order;
    a.total = grid.x * grid.y;
    uint8_t *bufs[2] = {static_cast<uint8_t *>(b0), static_cast<uint8_t *>(b1)};
    const int launches = fused + (steps - T * fused);
    for (int i = 0; i < launches; ++i) {
        a.src = bufs[i & 1];
        a.dst = bufs[(i + 1) & 1];
        void *args[] = {&a};
        hipError_t e = hipLaunchKernel((const void *)(i < fused ? fn2 : fn1), grid,
                                       dim3(t.threads), args, 0, s);
        if (e != hipSuccess)
            return hip_error(e, "step kernel launch");
    }
    return hip_error(hipGetLastError(), "step kernel launch");
}

StepFn pick_step(int map, int rule, int r, int threads, int flags)
{
    switch (map) {
    case MAP_LAMBDA: return pick_step_lambda(rule, r, threads, flags);
    case MAP_BB: return pick_step_bb(rule, r, threads, flags);
    case MAP_MFMA: return pick_step_mfma(rule, r, threads, flags);
    default: return nullptr;
    }
}

} // namespace fractal
