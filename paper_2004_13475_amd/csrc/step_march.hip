// step_march.hip -- instantiations and host launcher of the register-march
// step kernels (lambda and bounding-box maps).
#include <hip/hip_runtime.h>

#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

template <int MAP, int RULE, int R, int T, int FL>
static MarchFn march_fn()
{
    constexpr int HL = march_hl(RULE, T);
    if constexpr (MGeom<RULE, R, T, HL>::VALID && march_supported(RULE, T))
        return march_kernel<RULE, R, T, HL, MAP, FL, march_wpe(T), march_depth(RULE, T)>;
    else
        return nullptr;
}

template <int MAP, int RULE, int FL>
static MarchFn march_pick_rt(int r, int T)
{
    switch (r) {
#define FRACTAL_MARCH_R(RR)                                                                        \
    case RR:                                                                                       \
        switch (T) {                                                                               \
        case 1: return march_fn<MAP, RULE, RR, 1, FL>();                                           \
        case 2: return march_fn<MAP, RULE, RR, 2, FL>();                                           \
        case 4: return march_fn<MAP, RULE, RR, 4, FL>();                                           \
        case 8: return march_fn<MAP, RULE, RR, 8, FL>();                                           \
        case 16: return march_fn<MAP, RULE, RR, 16, FL>();                                           \
        default: return nullptr;                                                                   \
        }
        FRACTAL_MARCH_R(2)
        FRACTAL_MARCH_R(3)
        FRACTAL_MARCH_R(4)
        FRACTAL_MARCH_R(5)
        FRACTAL_MARCH_R(6)
        FRACTAL_MARCH_R(7)
#undef FRACTAL_MARCH_R
    default: return nullptr;
    }
}

template <int MAP>
static MarchFn march_pick_map(int rule, int r, int T, bool nt)
{
    if (rule == FRACTAL_RULE_CA)
        return nt ? march_pick_rt<MAP, RULE_CA, TILE_NT_STORE>(r, T)
                  : march_pick_rt<MAP, RULE_CA, 0>(r, T);
    return nt ? march_pick_rt<MAP, RULE_HEAT, TILE_NT_STORE>(r, T)
              : march_pick_rt<MAP, RULE_HEAT, 0>(r, T);
}

MarchFn pick_march(int map, int rule, int r, int T, bool nt)
{
    if (map == MAP_LAMBDA)
        return march_pick_map<MAP_LAMBDA>(rule, r, T, nt);
    if (map == MAP_BB)
        return march_pick_map<MAP_BB>(rule, r, T, nt);
    return nullptr;
}

int march_tiles_per_wave(int rule, int r, int T)
{
    const int S = rule == FRACTAL_RULE_CA ? 1 : 4;
    const int il = ((1 << r) * S) / 16;
    const int gl = il + 2 * march_hl(rule == FRACTAL_RULE_CA ? RULE_CA : RULE_HEAT, T);
    return (il >= 1 && gl <= 64) ? 64 / gl : 0;
}

// Bands per tile (log2): the fewest that give the chip about 2.5
// wavefronts per SIMD (fewer leave HBM latency exposed), keeping bands at
// least 4T rows high (the 2T halo rows each band re-reads stay cheap) and a
// multiple of the kernel's row period.
int march_band_log(int rule, int r, int T, uint64_t tiles)
{
    const uint64_t P = (uint64_t)march_tiles_per_wave(rule, r, T);
    const uint64_t want = 10u * 256u; // 2.5 wavefronts x 4 SIMDs x 256 CUs
    const int qr = march_row_period(rule == FRACTAL_RULE_CA ? RULE_CA : RULE_HEAT);
    const int hmin = 4 * T > qr ? 4 * T : qr;
    int b = 0;
    while (b < r && ((1 << r) >> (b + 1)) >= hmin && ((tiles << b) + P - 1) / P < want)
        ++b;
    return b;
}

// As many Tmax-step launches as fit, the rest in powers of two; if that
// count's parity differs from steps', the largest launch is split in two
// halves (the result then lands in buf[steps & 1]; splitting the largest
// costs least, since a launch's time grows with its step count).
void march_split(int steps, int Tmax, int (&counts)[kMaxListsPerItem])
{
    for (int j = 0; j < kMaxListsPerItem; ++j)
        counts[j] = 0;
    counts[0] = steps / Tmax;
    int total = counts[0];
    for (int j = 1; j < kMaxListsPerItem && (Tmax >> j) >= 1; ++j)
        if ((steps % Tmax) & (Tmax >> j)) {
            ++counts[j];
            ++total;
        }
    if ((total & 1) != (steps & 1)) {
        for (int j = 0; j < kMaxListsPerItem - 1 && (Tmax >> j) >= 2; ++j)
            if (counts[j] > 0) {
                --counts[j];
                counts[j + 1] += 2;
                break;
            }
    }
}

int launch_march(int map, int k, int rule, float alpha, void *b0, void *b1, int steps,
                 const fractal_tuning &t, hipStream_t s)
{
    const int Tmax = launch_steps_of(t.flags);
    const bool nt = (t.flags & FRACTAL_FLAG_NT_STORE) != 0;
    int counts[kMaxListsPerItem];
    march_split(steps, Tmax, counts);
    std::vector<int> plan;
    for (int j = 0; j < kMaxListsPerItem; ++j)
        for (int c = 0; c < counts[j]; ++c)
            plan.push_back(Tmax >> j);
    const int rb = k - t.r;
    const uint64_t tiles = map == MAP_BB ? (uint64_t)1 << (2 * rb) : pow3_u64(rb);
    MarchArgs a;
    a.k = k;
    a.alpha = alpha;
    a.rb = rb;
    a.order = t.order;
    a.total = (uint32_t)tiles;
    uint8_t *bufs[2] = {static_cast<uint8_t *>(b0), static_cast<uint8_t *>(b1)};
    const int wpg = t.threads / 64;
    for (size_t i = 0; i < plan.size(); ++i) {
        const int T = plan[i];
        MarchFn fn = pick_march(map, rule, t.r, T, nt);
        const int P = march_tiles_per_wave(rule, t.r, T);
        if (!fn || P < 1)
            return set_error(FRACTAL_E_INVAL, "no march kernel for rule %d r %d T %d", rule, t.r, T);
        a.band_log = march_band_log(rule, t.r, T, tiles);
        const uint64_t items = tiles << a.band_log;
        const uint64_t waves = (items + (uint64_t)P - 1) / (uint64_t)P;
        const uint64_t grid = (waves + (uint64_t)wpg - 1) / (uint64_t)wpg;
        a.src = bufs[i & 1];
        a.dst = bufs[(i + 1) & 1];
        void *args[] = {&a};
        hipError_t e = hipLaunchKernel((const void *)fn, dim3((unsigned)grid), dim3(t.threads),
                                       args, 0, s);
        if (e != hipSuccess)
            return hip_error(e, "march kernel launch");
    }
    return hip_error(hipGetLastError(), "march kernel launch");
}

} // namespace fractal
