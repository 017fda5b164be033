// compact.hip -- compact storage through lambda^-1 (the paper's closing
// future-work item): state sizes, pack / unpack between the n x n array and
// the compact layout, the seeded fill of a compact state, and the compact
// step entry point.  The layout is described in compact_march.hpp.
#include <hip/hip_runtime.h>

#include <vector>

#include "compact_march.hpp"
#include "internal.hpp"
#include "seed.hpp"

namespace fractal {

constexpr int kMaxCompactLevel = 20;
constexpr int kMaxCompactTileLevel = 18;

// One thread per (tile, 16-byte chunk column of the tile): the column's rho
// rows.  DIR 0: array -> compact; DIR 1: compact -> array.
template <int S, int DIR>
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *__restrict__ src,
                                                   uint8_t *__restrict__ dst, int k, int r,
                                                   uint64_t items)
{
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= items)
        return;
    const int rho = 1 << r;
    const int cpr = rho * S / 16; // chunk columns per tile row
    const uint64_t L = id / (uint64_t)cpr;
    const int q = (int)(id - L * (uint64_t)cpr);
    const TileXY t = lambda_lane((uint32_t)L, k - r, FRACTAL_ORDER_CURVE);
    const uint64_t n = 1ull << k;
    for (int j = 0; j < rho; ++j) {
        const uint64_t y = ((uint64_t)t.y << r) + (uint64_t)j;
        const uint64_t eoff = (y * n + ((uint64_t)t.x << r)) * S + (uint64_t)q * 16u;
        const uint64_t coff = ((L * (uint64_t)rho + (uint64_t)j) * (uint64_t)rho) * S +
                              (uint64_t)q * 16u;
        if constexpr (DIR == 0)
            *reinterpret_cast<u32x4 *>(dst + coff) = *reinterpret_cast<const u32x4 *>(src + eoff);
        else
            *reinterpret_cast<u32x4 *>(dst + eoff) = *reinterpret_cast<const u32x4 *>(src + coff);
    }
}

// Seeded fill of a compact state: the cells of every tile box get the value
// the seeded fill of the n x n array gives the same (x, y).
template <int RULE>
__global__ __launch_bounds__(256) void compact_seed_kernel(uint8_t *__restrict__ dst, int k,
                                                           int r, uint64_t items, uint64_t base)
{
    constexpr int S = RULE == FRACTAL_RULE_CA ? 1 : 4;
    constexpr int CELLS = 16 / S;
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= items)
        return;
    const int rho = 1 << r;
    const int cpr = rho * S / 16;
    const uint64_t L = id / (uint64_t)cpr;
    const int q = (int)(id - L * (uint64_t)cpr);
    const TileXY t = lambda_lane((uint32_t)L, k - r, FRACTAL_ORDER_CURVE);
    const uint32_t x0 = (t.x << r) + (uint32_t)q * CELLS;
    for (int j = 0; j < rho; ++j) {
        const uint32_t y = (t.y << r) + (uint32_t)j;
        uint32_t w[4];
        if constexpr (S == 1) {
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                uint32_t word = 0u;
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    word |= seeded_cell<RULE>(base, x0 + 4 * qq + b, y, k) << (8 * b);
                w[qq] = word;
            }
        } else {
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                w[qq] = seeded_cell<RULE>(base, x0 + qq, y, k);
        }
        const uint64_t coff = ((L * (uint64_t)rho + (uint64_t)j) * (uint64_t)rho) * S +
                              (uint64_t)q * 16u;
        *reinterpret_cast<u32x4 *>(dst + coff) = u32x4{w[0], w[1], w[2], w[3]};
    }
}

static int check_compact(int k, int r, int rule, int kmax)
{
    if (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT)
        return set_error(FRACTAL_E_INVAL, "unknown rule %d", rule);
    if (r < 0 || r > kMaxR || k < r || k > kmax || k - r > kMaxCompactTileLevel)
        return set_error(FRACTAL_E_INVAL,
                         "compact storage needs 0 <= r <= %d, r <= k <= %d, k - r <= %d "
                         "(k=%d r=%d)", kMaxR, kmax, kMaxCompactTileLevel, k, r);
    if ((1 << r) * (int)cell_bytes(rule) < 16)
        return set_error(FRACTAL_E_INVAL, "compact storage needs tile rows of >= 16 bytes "
                         "(r >= %d for this rule)", rule == FRACTAL_RULE_CA ? 4 : 2);
    return FRACTAL_OK;
}

static size_t compact_size(int k, int r, int rule)
{
    return (size_t)pow3_u64(k - r) * ((size_t)1 << (2 * r)) * cell_bytes(rule);
}

static bool aligned16(const void *p) { return p && reinterpret_cast<uintptr_t>(p) % 16 == 0; }

static int launch_items(int k, int r, int rule, uint64_t *items, unsigned *grid)
{
    const int cpr = (1 << r) * (int)cell_bytes(rule) / 16;
    *items = pow3_u64(k - r) * (uint64_t)cpr;
    const uint64_t g = (*items + 255) / 256;
    if (g > 0x7FFFFFFFull)
        return set_error(FRACTAL_E_INVAL, "grid too large");
    *grid = (unsigned)g;
    return FRACTAL_OK;
}

} // namespace fractal

using namespace fractal;

extern "C" {

int fractal_compact_bytes(int k, int r, int rule, size_t *bytes)
{
    if (!bytes)
        return set_error(FRACTAL_E_INVAL, "null output");
    int rc = check_compact(k, r, rule, kMaxCompactLevel);
    if (rc)
        return rc;
    *bytes = compact_size(k, r, rule);
    return FRACTAL_OK;
}

static int pack_entry(int k, int r, int rule, const void *src, void *dst, void *stream, int dir)
{
    int rc = check_compact(k, r, rule, kMaxStepLevel);
    if (rc)
        return rc;
    if (!aligned16(src) || !aligned16(dst))
        return set_error(FRACTAL_E_INVAL, "buffers must be non-null and 16-byte aligned");
    uint64_t items;
    unsigned grid;
    if ((rc = launch_items(k, r, rule, &items, &grid)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint8_t *a = static_cast<const uint8_t *>(src);
    uint8_t *b = static_cast<uint8_t *>(dst);
    if (rule == FRACTAL_RULE_CA) {
        if (dir == 0)
            hipLaunchKernelGGL((pack_kernel<1, 0>), dim3(grid), dim3(256), 0, s, a, b, k, r, items);
        else
            hipLaunchKernelGGL((pack_kernel<1, 1>), dim3(grid), dim3(256), 0, s, a, b, k, r, items);
    } else {
        if (dir == 0)
            hipLaunchKernelGGL((pack_kernel<4, 0>), dim3(grid), dim3(256), 0, s, a, b, k, r, items);
        else
            hipLaunchKernelGGL((pack_kernel<4, 1>), dim3(grid), dim3(256), 0, s, a, b, k, r, items);
    }
    return hip_error(hipGetLastError(), "pack kernel launch");
}

int fractal_pack(int k, int r, int rule, const void *d_embedded, void *d_compact, void *stream)
{
    return pack_entry(k, r, rule, d_embedded, d_compact, stream, 0);
}

int fractal_unpack(int k, int r, int rule, const void *d_compact, void *d_embedded, void *stream)
{
    return pack_entry(k, r, rule, d_compact, d_embedded, stream, 1);
}

int fractal_compact_seed_fill(int k, int r, int rule, uint32_t stream_id, void *d_compact,
                              void *stream)
{
    int rc = check_compact(k, r, rule, kMaxCompactLevel);
    if (rc)
        return rc;
    if (!aligned16(d_compact))
        return set_error(FRACTAL_E_INVAL, "buffer must be non-null and 16-byte aligned");
    uint64_t items;
    unsigned grid;
    if ((rc = launch_items(k, r, rule, &items, &grid)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t base = (uint64_t)stream_id << 32;
    uint8_t *b = static_cast<uint8_t *>(d_compact);
    if (rule == FRACTAL_RULE_CA)
        hipLaunchKernelGGL(compact_seed_kernel<FRACTAL_RULE_CA>, dim3(grid), dim3(256), 0, s, b, k,
                           r, items, base);
    else
        hipLaunchKernelGGL(compact_seed_kernel<FRACTAL_RULE_HEAT>, dim3(grid), dim3(256), 0, s, b,
                           k, r, items, base);
    return hip_error(hipGetLastError(), "compact seed launch");
}

int fractal_compact_step(int k, int r, int rule, float alpha, void *d_c0, void *d_c1, int steps,
                         int flags, void *stream)
{
    int rc = check_compact(k, r, rule, kMaxCompactLevel);
    if (rc)
        return rc;
    if (rule == FRACTAL_RULE_HEAT && !(alpha > 0.0f && alpha <= 0.25f))
        return set_error(FRACTAL_E_INVAL, "heat needs 0 < alpha <= 0.25");
    if (steps < 0)
        return set_error(FRACTAL_E_INVAL, "steps must be >= 0");
    if (!aligned16(d_c0) || !aligned16(d_c1))
        return set_error(FRACTAL_E_INVAL, "buffers must be non-null and 16-byte aligned");
    const size_t bytes = compact_size(k, r, rule);
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(d_c0), p1 = reinterpret_cast<uintptr_t>(d_c1);
    if (p0 < p1 + bytes && p1 < p0 + bytes)
        return set_error(FRACTAL_E_INVAL, "the two compact buffers overlap");
    const int fuse = flags & kFuseFlags;
    const bool block = (flags & FRACTAL_FLAG_BLOCK) != 0;
    if ((flags & ~(FRACTAL_FLAG_NT_STORE | FRACTAL_FLAG_SEGMENTS | FRACTAL_FLAG_MARCH |
                   FRACTAL_FLAG_BLOCK | kFuseFlags)) ||
        (fuse & (fuse - 1)) || ((fuse & kDeepFlags) && !block) ||
        (block && (flags & FRACTAL_FLAG_MARCH)))
        return set_error(FRACTAL_E_INVAL, "unknown flags 0x%x", flags);
    if (block && r != 6)
        return set_error(FRACTAL_E_INVAL, "the block engine takes compact states of 64 x 64 tiles (r = 6)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // 64 x 64 tiles: the block engine (by default with 36 steps per launch)
    if (block || (flags == 0 && r == 6)) {
        const int cap = block ? launch_steps_of(flags) : 36;
        return launch_compact_block(k, rule, alpha, d_c0, d_c1, steps, cap,
                                    (flags & FRACTAL_FLAG_NT_STORE) != 0, s);
    }
    int Tmax;
    bool nt;
    if (flags == 0) {
        // default: the longest launch the tile allows, up to 16 (automaton,
        // level >= 15) or 8 steps; non-temporal stores from level 15
        nt = k >= 15;
        Tmax = (rule == FRACTAL_RULE_CA && k >= 15) ? 16 : 8;
        while (Tmax > 1 && !(rule == FRACTAL_RULE_CA ? pick_compact_ca(r, Tmax, nt)
                                                     : pick_compact_heat(r, Tmax, nt)))
            Tmax /= 2;
    } else {
        nt = (flags & FRACTAL_FLAG_NT_STORE) != 0;
        Tmax = launch_steps_of(flags);
        if (!(rule == FRACTAL_RULE_CA ? pick_compact_ca(r, Tmax, nt) : pick_compact_heat(r, Tmax, nt)))
            return set_error(FRACTAL_E_INVAL,
                             "no compact kernel for rule %d r %d with %d steps per launch "
                             "(steps and halo must fit in one tile)", rule, r, Tmax);
    }
    if (steps == 0)
        return FRACTAL_OK;
    int counts[kMaxListsPerItem];
    march_split(steps, Tmax, counts);
    const int rb = k - r;
    CompactArgs a;
    a.k = k;
    a.alpha = alpha;
    a.rb = rb;
    a.total = (uint32_t)pow3_u64(rb);
    uint8_t *bufs[2] = {static_cast<uint8_t *>(d_c0), static_cast<uint8_t *>(d_c1)};
    int launch = 0;
    for (int j = 0; j < kMaxListsPerItem; ++j) {
        const int T = Tmax >> j;
        for (int c = 0; c < counts[j]; ++c, ++launch) {
            CompactFn fn = rule == FRACTAL_RULE_CA ? pick_compact_ca(r, T, nt)
                                                   : pick_compact_heat(r, T, nt);
            const int P = march_tiles_per_wave(rule, r, T);
            if (!fn || P < 1)
                return set_error(FRACTAL_E_INVAL, "no compact kernel for r %d T %d", r, T);
            a.band_log = march_band_log(rule, r, T, a.total);
            const uint64_t waves = (((uint64_t)a.total << a.band_log) + (uint64_t)P - 1) / (uint64_t)P;
            const uint64_t grid = (waves + 3) / 4;
            a.src = bufs[launch & 1];
            a.dst = bufs[(launch + 1) & 1];
            void *args[] = {&a};
            hipError_t e = hipLaunchKernel((const void *)fn, dim3((unsigned)grid), dim3(256), args, 0, s);
            if (e != hipSuccess)
                return hip_error(e, "compact march launch");
        }
    }
    return hip_error(hipGetLastError(), "compact march launch");
}

} // extern "C"
