// step_kernels.hip -- lambda(omega) map kernels and the lambda / bounding-box
// step kernels for gfx950, with their host launchers.
#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "device_tile.hpp"
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

// ------------------------------------------------------------------ steps
struct LaunchArgs {
    StepParams p;
    int rb;         // block-space level k - r
    int order;      // FRACTAL_ORDER_*
    uint32_t total; // workgroups in the grid
};

// One workgroup per tile.  lambda maps: the grid is the compact 3^ceil(rb/2)
// x 3^floor(rb/2) orthotope.  Bounding box: the grid is n_b x n_b and a
// workgroup on an empty tile returns before touching memory.
template <int RULE, int R, int NT, int MAP, int FL>
__global__ __launch_bounds__(NT) void step_kernel(LaunchArgs a)
{
    __shared__ __align__(16) uint8_t lds[Geom<RULE, R>::LDS_BYTES];
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
    tile_step<RULE, R, NT, FL>(lds, a.p, t.x << R, t.y << R);
}

typedef void (*StepFn)(LaunchArgs);

template <int MAP, int RULE, int NT, int FL>
static StepFn pick_r(int r)
{
    switch (r) {
    case 0: return step_kernel<RULE, 0, NT, MAP, FL>;
    case 1: return step_kernel<RULE, 1, NT, MAP, FL>;
    case 2: return step_kernel<RULE, 2, NT, MAP, FL>;
    case 3: return step_kernel<RULE, 3, NT, MAP, FL>;
    case 4: return step_kernel<RULE, 4, NT, MAP, FL>;
    case 5: return step_kernel<RULE, 5, NT, MAP, FL>;
    case 6: return step_kernel<RULE, 6, NT, MAP, FL>;
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
static StepFn pick_flags(int rule, int r, int threads, int flags)
{
    switch (flags & 3) {
    case 0: return pick_rule<MAP, 0>(rule, r, threads);
    case 1: return pick_rule<MAP, 1>(rule, r, threads);
    case 2: return pick_rule<MAP, 2>(rule, r, threads);
    default: return pick_rule<MAP, 3>(rule, r, threads);
    }
}

static StepFn pick(int map, int rule, int r, int threads, int flags)
{
    switch (map) {
    case MAP_LAMBDA: return pick_flags<MAP_LAMBDA>(rule, r, threads, flags);
    case MAP_BB: return pick_flags<MAP_BB>(rule, r, threads, flags);
    case MAP_MFMA: return pick_flags<MAP_MFMA>(rule, r, threads, flags);
    default: return nullptr;
    }
}

int launch_steps(int map, int k, int rule, float alpha, void *b0, void *b1,
                 int steps, const fractal_tuning &t, hipStream_t s)
{
    StepFn fn = pick(map, rule, t.r, t.threads, t.flags);
    if (!fn)
        return set_error(FRACTAL_E_INVAL, "no kernel for map %d rule %d r %d threads %d",
                         map, rule, t.r, t.threads);
    const int rb = k - t.r;
    dim3 grid;
    if (map == MAP_BB)
        grid = dim3(1u << rb, 1u << rb);
    else
        grid = dim3((unsigned)pow3_u64((rb + 1) / 2), (unsigned)pow3_u64(rb / 2));
    LaunchArgs a;
    a.p.k = k;
    a.p.alpha = alpha;
    a.rb = rb;
    a.order = t.order;
    a.total = grid.x * grid.y;
    uint8_t *bufs[2] = {static_cast<uint8_t *>(b0), static_cast<uint8_t *>(b1)};
    for (int i = 0; i < steps; ++i) {
        a.p.src = bufs[i & 1];
        a.p.dst = bufs[(i + 1) & 1];
        void *args[] = {&a};
        hipError_t e = hipLaunchKernel((const void *)fn, grid, dim3(t.threads), args, 0, s);
        if (e != hipSuccess)
            return hip_error(e, "step kernel launch");
    }
    return hip_error(hipGetLastError(), "step kernel launch");
}

} // namespace fractal
