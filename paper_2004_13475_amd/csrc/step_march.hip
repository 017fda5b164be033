// step_march.hip -- host launcher of the register-march step kernels
// (lambda and bounding-box maps); the kernels are instantiated per rule in
// step_march_ca.hip and step_march_heat.hip, those of 10 and 12 steps in
// step_march_mid_ca.hip and step_march_mid_heat.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

MarchFn pick_march_ca(int map, int r, int T, bool nt, bool alt);
MarchFn pick_march_heat(int map, int r, int T, bool nt, bool alt);

MarchFn pick_march(int map, int rule, int r, int T, bool nt, bool alt)
{
    return rule == FRACTAL_RULE_CA ? pick_march_ca(map, r, T, nt, alt)
                                   : pick_march_heat(map, r, T, nt, alt);
}

MarchFn pick_march_mid_ca(int r, int T, bool nt);
MarchFn pick_march_mid_heat(int r, int T, bool nt);

MarchFn pick_march_mid(int rule, int r, int T, bool nt)
{
    return rule == FRACTAL_RULE_CA ? pick_march_mid_ca(r, T, nt) : pick_march_mid_heat(r, T, nt);
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
// count's parity differs from steps' (and even_parity asks for it), the
// largest launch is split in two halves (the result then lands in
// buf[steps & 1]; splitting the largest costs least, since a launch's time
// grows with its step count).
void march_split(int steps, int Tmax, int (&counts)[kMaxListsPerItem], bool even_parity)
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
    if (even_parity && (total & 1) != (steps & 1)) {
        for (int j = 0; j < kMaxListsPerItem - 1 && (Tmax >> j) >= 2; ++j)
            if (counts[j] > 0) {
                --counts[j];
                counts[j + 1] += 2;
                break;
            }
    }
}

// Launch sizes of a sixteen-step lambda tuning: a launch reads and writes
// the state's member segments whatever its step count, so a short launch
// costs about as much as a launch of ten steps (the level-16 automaton and
// heat launches of 1 to 4 steps take 55-65% of a sixteen-step one, those of
// ten steps 80%).  With a cost of max(10, T) per launch of T steps, the plan
// is the cheapest set of launch sizes from `sizes` that adds up to `steps`
// with a launch count of the parity of `steps` (the result lands in
// buf[steps & 1]): 20 steps run as 10 + 10 rather than 16 + 4.  All but the
// last 48-63 steps run as sixteen-step launches; the rest is a small exact
// search.
static void march_plan_cost(int steps, const std::vector<int> &sizes, std::vector<int> &plan)
{
    if (steps <= 0)
        return;
    const int q = steps / 16 > 3 ? steps / 16 - 3 : 0;
    for (int i = 0; i < q; ++i)
        plan.push_back(16);
    const int rem = steps - 16 * q;
    const int INF = 1 << 28;
    // best[s][p]: least cost of launches adding up to s steps, count parity p
    std::vector<int> best(2 * (rem + 1), INF), pick(2 * (rem + 1), 0);
    best[0] = 0;
    for (int t = 1; t <= rem; ++t)
        for (int p = 0; p < 2; ++p)
            for (int T : sizes) {
                if (T > t || best[2 * (t - T) + (p ^ 1)] >= INF)
                    continue;
                const int c = best[2 * (t - T) + (p ^ 1)] + (T > 10 ? T : 10) * 64 + 1;
                if (c < best[2 * t + p]) {
                    best[2 * t + p] = c;
                    pick[2 * t + p] = T;
                }
            }
    int p = (steps & 1) ^ (q & 1), t = rem;
    std::vector<int> tail;
    while (t > 0 && best[2 * t + p] < INF) {
        const int T = pick[2 * t + p];
        tail.push_back(T);
        t -= T;
        p ^= 1;
    }
    std::sort(tail.begin(), tail.end(), [](int x, int y) { return x > y; });
    plan.insert(plan.end(), tail.begin(), tail.end());
}

// The runtime loads a source file's kernels onto a device the first time
// one of them runs (about a millisecond each).  A call's launches can use
// the kernels of several sources (the 10- and 12-step kernels sit apart
// from the others), so the first call on a device loads every march source
// of both rules up front instead of in the middle of a run.
static void preload_march_code()
{
    static std::mutex mu;
    static bool done[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return;
    std::lock_guard<std::mutex> lock(mu);
    if (done[dev])
        return;
    done[dev] = true;
    for (int rule : {FRACTAL_RULE_CA, FRACTAL_RULE_HEAT}) {
        const MarchFn fns[] = {pick_march(MAP_LAMBDA, rule, 4, 1, false, false),
                               pick_march_mid(rule, 4, 10, false)};
        for (MarchFn fn : fns) {
            hipFuncAttributes attr;
            if (fn)
                (void)hipFuncGetAttributes(&attr, (const void *)fn); // loads its code object
        }
    }
}

int launch_march(int map, int k, int rule, float alpha, void *b0, void *b1, int steps,
                 const fractal_tuning &t, hipStream_t s)
{
    preload_march_code();
    const int Tmax = launch_steps_of(t.flags);
    const bool nt = (t.flags & FRACTAL_FLAG_NT_STORE) != 0;
    const bool alt = (t.flags & FRACTAL_FLAG_OCC_ALT) != 0;
    std::vector<int> plan;
    if (map == MAP_LAMBDA && Tmax == 16) {
        std::vector<int> sizes{16};
        for (int T : {12, 10})
            if (pick_march_mid(rule, t.r, T, nt))
                sizes.push_back(T);
        for (int T : {8, 4, 2, 1})
            sizes.push_back(T);
        march_plan_cost(steps, sizes, plan);
    } else {
        int counts[kMaxListsPerItem];
        march_split(steps, Tmax, counts);
        for (int j = 0; j < kMaxListsPerItem; ++j)
            for (int c = 0; c < counts[j]; ++c)
                plan.push_back(Tmax >> j);
    }
    const int rb = k - t.r;
    const uint64_t tiles = map == MAP_BB ? (uint64_t)1 << (2 * rb) : pow3_u64(rb);
    MarchArgs a;
    a.k = k;
    a.alpha = alpha;
    a.rb = rb;
    a.order = t.order;
    a.total = (uint32_t)tiles;
    a.stack_log = map == MAP_LAMBDA ? stack_log_of(t.flags) : 0;
    if (a.stack_log > rb)
        a.stack_log = rb;
    a.stack_waves = 0u;
    uint8_t *bufs[2] = {static_cast<uint8_t *>(b0), static_cast<uint8_t *>(b1)};
    const int wpg = t.threads / 64;
    for (size_t i = 0; i < plan.size(); ++i) {
        const int T = plan[i];
        MarchFn fn = (T == 10 || T == 12) ? pick_march_mid(rule, t.r, T, nt)
                                          : pick_march(map, rule, t.r, T, nt, alt);
        const int P = march_tiles_per_wave(rule, t.r, T);
        if (!fn || P < 1)
            return set_error(FRACTAL_E_INVAL, "no march kernel for rule %d r %d T %d", rule, t.r, T);
        uint64_t waves = 0;
        if (a.stack_log > 0) {
            a.band_log = 0;
            // groups of P blocks of 2^c x 2^c tiles, 1 + (3^c - 1) / 2 wavefronts each
            const uint64_t groups = (pow3_u64(rb - a.stack_log) + (uint64_t)P - 1) / (uint64_t)P;
            waves = groups * (1u + (pow3_u64(a.stack_log) - 1u) / 2u);
            a.stack_waves = (uint32_t)waves;
        } else {
            a.band_log = march_band_log(rule, t.r, T, tiles);
            const uint64_t items = tiles << a.band_log;
            waves = (items + (uint64_t)P - 1) / (uint64_t)P;
        }
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
