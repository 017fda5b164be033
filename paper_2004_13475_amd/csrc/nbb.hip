// nbb.hip -- the general NBB family (Section 3, Table 1): any fractal given
// by k replicas per level on an s x s grid, replica beta at offset
// H[beta] = (tau_x, tau_y).  lambda(omega) of Theorem 1 for any such table,
// and tests SW, RD and the automaton over tiles of side s^r reached through
// lambda or the bounding box.
//
// With s = 2 and 0/1 offsets the per-level offsets of lambda fill disjoint
// bits, which the gasket kernels turn into two ballots; in general they do
// not, so here every wavefront sums the levels' offsets by a butterfly over
// its lanes -- the parallel reduction of Theorem 1's proof, done in
// registers.
#include <hip/hip_runtime.h>

#include "device_map.hpp"
#include "internal.hpp"

namespace fractal {

constexpr int kNbbMaxTile = 128; // tile side s^r

struct NbbDev {
    int k, s;
    uint8_t tx[FRACTAL_NBB_MAX_K], ty[FRACTAL_NBB_MAX_K];
    int8_t inv[64];    // replica index of grid cell dy * s + dx, or -1
    uint64_t pos_mask; // bit dy * s + dx set for the replica cells
};

struct NbbArgs {
    NbbDev f;
    const uint8_t *src;
    uint8_t *dst;
    uint64_t *slots;
    int level; // n = s^level
    int r;     // tile side b = s^r
    int rb;    // level - r
    uint32_t n, b, nb;
    uint32_t gx; // columns of the compact grid (k^ceil(rb/2))
    uint32_t value;
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
        v += (uint32_t)__builtin_amdgcn_ds_bpermute((int)((lane_id() ^ (uint32_t)off) << 2),
                                                    (int)v);
    return v;
}

// Theorem 1: lane j < rb evaluates level mu = j + 1: beta_mu is base-k digit
// ceil(mu/2) - 1 of omega_x (odd mu) or omega_y (even mu), tau = H[beta], and
// the level's offset is tau * s^(mu-1); the wavefront sums the offsets.
// Uniform result; all 64 lanes must call it.
__device__ __forceinline__ TileXY nbb_lambda(const NbbDev &f, uint32_t wx, uint32_t wy, int rb)
{
    const uint32_t j = lane_id();
    uint32_t dx = 0u, dy = 0u;
    if (j < (uint32_t)rb) {
        uint32_t v = (j & 1u) ? wy : wx;
        for (uint32_t q = 0; q < (j >> 1); ++q)
            v /= (uint32_t)f.k;
        const uint32_t beta = v % (uint32_t)f.k;
        uint32_t p = 1u;
        for (uint32_t q = 0; q < j; ++q)
            p *= (uint32_t)f.s;
        dx = (uint32_t)f.tx[beta] * p;
        dy = (uint32_t)f.ty[beta] * p;
    }
    return TileXY{wave_sum_u32(dx), wave_sum_u32(dy)};
}

// Is (x, y) (coordinates at a level of `digits` base-s digits) a member?
__device__ __forceinline__ bool nbb_member(const NbbDev &f, uint32_t x, uint32_t y, int digits)
{
    bool m = true;
    for (int d = 0; d < digits; ++d) {
        const uint32_t qx = x / (uint32_t)f.s, qy = y / (uint32_t)f.s;
        const uint32_t cx = x - qx * (uint32_t)f.s, cy = y - qy * (uint32_t)f.s;
        m = m && ((f.pos_mask >> (cy * (uint32_t)f.s + cx)) & 1ull);
        x = qx;
        y = qy;
    }
    return m;
}

// Row-major slot of the compact grid cell omega whose lambda is block (X, Y)
// (the inverse map, digit by digit), for deterministic per-tile sums.
__device__ __forceinline__ uint32_t nbb_slot(const NbbDev &f, uint32_t X, uint32_t Y, int rb,
                                             uint32_t gx)
{
    uint32_t wx = 0u, wy = 0u, px = 1u, py = 1u;
    for (int j = 0; j < rb; ++j) {
        const uint32_t qx = X / (uint32_t)f.s, qy = Y / (uint32_t)f.s;
        const uint32_t cx = X - qx * (uint32_t)f.s, cy = Y - qy * (uint32_t)f.s;
        const uint32_t beta = (uint32_t)f.inv[cy * (uint32_t)f.s + cx];
        if ((j & 1) == 0) {
            wx += beta * px;
            px *= (uint32_t)f.k;
        } else {
            wy += beta * py;
            py *= (uint32_t)f.k;
        }
        X = qx;
        Y = qy;
    }
    return wy * gx + wx;
}

enum : int { NBB_SW = 0, NBB_RD = 1, NBB_CA = 2 };

// One workgroup per tile: the compact grid (lambda, map 0) or all n_b x n_b
// blocks (BB, map 1; a workgroup on an empty block returns at once).
template <int MAP, int OP>
__global__ __launch_bounds__(256) void nbb_tile_kernel(NbbArgs a)
{
    __shared__ uint8_t vals[(kNbbMaxTile + 2) * (kNbbMaxTile + 2)];
    __shared__ uint8_t memb[kNbbMaxTile * kNbbMaxTile];
    __shared__ uint64_t part[256];
    uint32_t X, Y, slot = 0u;
    if constexpr (MAP == MAP_BB) {
        X = blockIdx.x;
        Y = blockIdx.y;
        if (!nbb_member(a.f, X, Y, a.rb))
            return; // empty block
        if constexpr (OP == NBB_RD)
            slot = nbb_slot(a.f, X, Y, a.rb, a.gx);
    } else {
        const TileXY t = nbb_lambda(a.f, blockIdx.x, blockIdx.y, a.rb);
        X = t.x;
        Y = t.y;
        slot = blockIdx.y * a.gx + blockIdx.x;
    }
    const uint32_t b = a.b, tid = threadIdx.x;
    const uint64_t x0 = (uint64_t)X * b, y0 = (uint64_t)Y * b;
    const uint32_t cells = b * b;
    // the pattern inside every non-empty tile is the level-r fractal
    for (uint32_t c = tid; c < cells; c += blockDim.x)
        memb[c] = nbb_member(a.f, c % b, c / b, a.r) ? 1u : 0u;
    if constexpr (OP == NBB_CA) {
        const uint32_t w = b + 2;
        for (uint32_t c = tid; c < w * w; c += blockDim.x) {
            const int64_t x = (int64_t)x0 + (int64_t)(c % w) - 1;
            const int64_t y = (int64_t)y0 + (int64_t)(c / w) - 1;
            uint8_t v = 0u;
            if (x >= 0 && y >= 0 && x < (int64_t)a.n && y < (int64_t)a.n)
                v = a.src[(uint64_t)y * a.n + (uint64_t)x];
            vals[c] = v;
        }
    }
    __syncthreads();
    uint64_t acc = 0u;
    for (uint32_t c = tid; c < cells; c += blockDim.x) {
        const uint32_t i = c % b, j = c / b;
        const uint64_t off = (y0 + j) * a.n + x0 + i;
        if constexpr (OP == NBB_SW) {
            if (memb[c])
                a.dst[off] = (uint8_t)a.value;
        } else if constexpr (OP == NBB_RD) {
            if (memb[c])
                acc += a.src[off];
        } else {
            const uint32_t w = b + 2;
            const uint32_t q = (j + 1) * w + (i + 1);
            uint8_t out = 0u;
            if (memb[c]) {
                // off-fractal cells hold 0, so the plain Moore sum counts
                // fractal neighbours only
                const uint32_t cnt = vals[q - w - 1] + vals[q - w] + vals[q - w + 1] +
                                     vals[q - 1] + vals[q + 1] + vals[q + w - 1] + vals[q + w] +
                                     vals[q + w + 1];
                out = (cnt == 3u || (vals[q] && cnt == 2u)) ? 1u : 0u;
            }
            a.dst[off] = out;
        }
    }
    if constexpr (OP == NBB_RD) {
        part[tid] = acc;
        __syncthreads();
        for (uint32_t s = blockDim.x >> 1; s > 0; s >>= 1) {
            if (tid < s)
                part[tid] += part[tid + s];
            __syncthreads();
        }
        if (tid == 0)
            a.slots[slot] = part[0];
    }
}

// lambda(omega) for every omega of the compact grid, one wavefront each.
__global__ __launch_bounds__(256) void nbb_map_kernel(NbbDev f, uint32_t *xy, int rb, uint32_t gx,
                                                      uint64_t total)
{
    const uint64_t wave = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint64_t stride = (uint64_t)gridDim.x * 4u;
    for (uint64_t i = wave; i < total; i += stride) {
        const TileXY t = nbb_lambda(f, (uint32_t)(i % gx), (uint32_t)(i / gx), rb);
        if ((threadIdx.x & 63u) == 0u) {
            xy[2 * i + 0] = t.x;
            xy[2 * i + 1] = t.y;
        }
    }
}

static uint64_t ipow(uint64_t b, int e)
{
    uint64_t p = 1;
    for (int i = 0; i < e; ++i)
        p *= b;
    return p;
}

static int check_nbb(const fractal_nbb *f, NbbDev *d)
{
    if (!f)
        return set_error(FRACTAL_E_INVAL, "null fractal");
    if (f->s < 2 || f->s > 8 || f->k < 1 || f->k > f->s * f->s || f->k > FRACTAL_NBB_MAX_K)
        return set_error(FRACTAL_E_INVAL, "need 2 <= s <= 8, 1 <= k <= min(s^2, %d) (k=%d s=%d)",
                         FRACTAL_NBB_MAX_K, f->k, f->s);
    d->k = f->k;
    d->s = f->s;
    d->pos_mask = 0;
    for (int i = 0; i < 64; ++i)
        d->inv[i] = -1;
    for (int i = 0; i < FRACTAL_NBB_MAX_K; ++i) {
        d->tx[i] = i < f->k ? f->tau_x[i] : 0;
        d->ty[i] = i < f->k ? f->tau_y[i] : 0;
    }
    for (int i = 0; i < f->k; ++i) {
        if (f->tau_x[i] >= f->s || f->tau_y[i] >= f->s)
            return set_error(FRACTAL_E_INVAL, "replica %d offset outside [0, s)", i);
        const int p = f->tau_y[i] * f->s + f->tau_x[i];
        if (d->inv[p] >= 0)
            return set_error(FRACTAL_E_INVAL, "replicas %d and %d overlap", d->inv[p], i);
        d->inv[p] = (int8_t)i;
        d->pos_mask |= 1ull << p;
    }
    return FRACTAL_OK;
}

static int nbb_setup(const fractal_nbb *f, int level, int r, NbbArgs *a)
{
    int rc = check_nbb(f, &a->f);
    if (rc)
        return rc;
    if (r < 0 || level < r)
        return set_error(FRACTAL_E_INVAL, "need 0 <= r <= level (level=%d r=%d)", level, r);
    const uint64_t n = ipow((uint64_t)f->s, level);
    const uint64_t b = ipow((uint64_t)f->s, r);
    if (n > 65536 || n * n > (1ull << 32))
        return set_error(FRACTAL_E_INVAL, "n = s^level must be <= 65536 with n^2 <= 2^32");
    if (b > (uint64_t)kNbbMaxTile)
        return set_error(FRACTAL_E_INVAL, "tile side s^r must be <= %d", kNbbMaxTile);
    const int rb = level - r;
    const uint64_t gx = ipow((uint64_t)f->k, (rb + 1) / 2), gy = ipow((uint64_t)f->k, rb / 2);
    if (gx > 0x7FFFFFFFull || gy > 65535ull)
        return set_error(FRACTAL_E_INVAL, "compact grid %llu x %llu beyond launch limits",
                         (unsigned long long)gx, (unsigned long long)gy);
    a->level = level;
    a->r = r;
    a->rb = rb;
    a->n = (uint32_t)n;
    a->b = (uint32_t)b;
    a->nb = (uint32_t)(n / b);
    a->gx = (uint32_t)gx;
    return FRACTAL_OK;
}

template <int OP>
static int nbb_launch(int map, NbbArgs &a, hipStream_t s)
{
    if (map != MAP_LAMBDA && map != MAP_BB)
        return set_error(FRACTAL_E_INVAL, "map %d: lambda (0) or BB (1)", map);
    if (map == MAP_BB && a.nb > 65535u)
        return set_error(FRACTAL_E_INVAL, "bounding box of %u x %u blocks beyond launch limits",
                         a.nb, a.nb);
    dim3 grid;
    if (map == MAP_BB)
        grid = dim3(a.nb, a.nb);
    else
        grid = dim3(a.gx, (unsigned)ipow((uint64_t)a.f.k, a.rb / 2));
    const unsigned threads = a.b * a.b >= 256 ? 256 : 64;
    if (map == MAP_BB)
        hipLaunchKernelGGL((nbb_tile_kernel<MAP_BB, OP>), grid, dim3(threads), 0, s, a);
    else
        hipLaunchKernelGGL((nbb_tile_kernel<MAP_LAMBDA, OP>), grid, dim3(threads), 0, s, a);
    return hip_error(hipGetLastError(), "NBB kernel launch");
}

} // namespace fractal

using namespace fractal;

extern "C" {

int fractal_nbb_builtin(int which, fractal_nbb *out)
{
    if (!out)
        return set_error(FRACTAL_E_INVAL, "null output");
    // replica cells (dx, dy) in row-major order of the s x s grid
    static const struct {
        int k, s;
        const char *cells; // s*s characters, row by row, '#' = replica
    } table[] = {
        {3, 2, "#." "##"},           // gasket, the paper's H = {(0,0), (0,1), (1,1)}
        {8, 3, "###" "#.#" "###"},   // Sierpinski carpet
        {5, 3, ".#." "###" ".#."},   // Vicsek fractal
        {5, 3, "#.#" ".#." "#.#"},   // X-fractal
        {7, 3, "#.#" "###" "#.#"},   // H-fractal
        {2, 3, "#.#" "..." "..."},   // Cantor set (on one row)
    };
    if (which < 0 || which >= (int)(sizeof(table) / sizeof(table[0])))
        return set_error(FRACTAL_E_INVAL, "unknown built-in fractal %d", which);
    fractal_nbb f{};
    f.k = table[which].k;
    f.s = table[which].s;
    int i = 0;
    for (int y = 0; y < f.s; ++y)
        for (int x = 0; x < f.s; ++x)
            if (table[which].cells[y * f.s + x] == '#') {
                f.tau_x[i] = (uint8_t)x;
                f.tau_y[i] = (uint8_t)y;
                ++i;
            }
    if (which == FRACTAL_NBB_GASKET) {
        // the paper's numbering: beta 0, 1, 2 -> (0,0), (0,1), (1,1)
        f.tau_x[0] = 0; f.tau_y[0] = 0;
        f.tau_x[1] = 0; f.tau_y[1] = 1;
        f.tau_x[2] = 1; f.tau_y[2] = 1;
    }
    *out = f;
    return FRACTAL_OK;
}

int fractal_nbb_lambda_map(const fractal_nbb *f, int rb, uint32_t *d_xy, void *stream)
{
    NbbDev d;
    int rc = check_nbb(f, &d);
    if (rc)
        return rc;
    if (!d_xy)
        return set_error(FRACTAL_E_INVAL, "null output buffer");
    if (rb < 0 || rb > 30 || ipow((uint64_t)f->s, rb) > (1ull << 31) ||
        ipow((uint64_t)f->k, rb) > (1ull << 31))
        return set_error(FRACTAL_E_INVAL, "level %d out of range", rb);
    const uint64_t gx = ipow((uint64_t)f->k, (rb + 1) / 2), gy = ipow((uint64_t)f->k, rb / 2);
    const uint64_t total = gx * gy;
    const uint64_t want = (total + 3) / 4;
    const unsigned grid = (unsigned)(want < (1u << 20) ? want : (1u << 20));
    hipLaunchKernelGGL(nbb_map_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                       d, d_xy, rb, (uint32_t)gx, total);
    return hip_error(hipGetLastError(), "NBB map launch");
}

int fractal_nbb_single_write(const fractal_nbb *f, int map, int level, int r, uint32_t value,
                             void *d_buf, void *stream)
{
    NbbArgs a{};
    int rc = nbb_setup(f, level, r, &a);
    if (rc)
        return rc;
    if (!d_buf)
        return set_error(FRACTAL_E_INVAL, "null buffer");
    a.dst = static_cast<uint8_t *>(d_buf);
    a.value = value & 0xFFu;
    return nbb_launch<NBB_SW>(map, a, static_cast<hipStream_t>(stream));
}

int fractal_nbb_reduce_workspace(const fractal_nbb *f, int level, int r, size_t *bytes)
{
    NbbArgs a{};
    int rc = nbb_setup(f, level, r, &a);
    if (rc)
        return rc;
    if (!bytes)
        return set_error(FRACTAL_E_INVAL, "null output");
    const uint64_t slots = (uint64_t)a.gx * ipow((uint64_t)f->k, a.rb / 2);
    *bytes = (size_t)(8 * reduce_tree_words(slots));
    return FRACTAL_OK;
}

int fractal_nbb_reduce(const fractal_nbb *f, int map, int level, int r, const void *d_buf,
                       void *d_work, size_t work_bytes, void *d_out, void *stream)
{
    NbbArgs a{};
    int rc = nbb_setup(f, level, r, &a);
    if (rc)
        return rc;
    size_t need = 0;
    if ((rc = fractal_nbb_reduce_workspace(f, level, r, &need)))
        return rc;
    if (!d_buf || !d_work || !d_out)
        return set_error(FRACTAL_E_INVAL, "null buffer, workspace or output");
    if (reinterpret_cast<uintptr_t>(d_work) % 8 || reinterpret_cast<uintptr_t>(d_out) % 8)
        return set_error(FRACTAL_E_INVAL, "workspace and output must be 8-byte aligned");
    if (work_bytes < need)
        return set_error(FRACTAL_E_INVAL, "workspace of %zu bytes, %zu needed", work_bytes, need);
    a.src = static_cast<const uint8_t *>(d_buf);
    a.slots = static_cast<uint64_t *>(d_work);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = nbb_launch<NBB_RD>(map, a, s)))
        return rc;
    const uint64_t slots = (uint64_t)a.gx * ipow((uint64_t)f->k, a.rb / 2);
    return launch_reduce_tree(a.slots, slots, d_out, false, s);
}

int fractal_nbb_ca_step(const fractal_nbb *f, int map, int level, int r, void *d_buf0,
                        void *d_buf1, int steps, void *stream)
{
    NbbArgs a{};
    int rc = nbb_setup(f, level, r, &a);
    if (rc)
        return rc;
    if (!d_buf0 || !d_buf1 || d_buf0 == d_buf1)
        return set_error(FRACTAL_E_INVAL, "need two distinct buffers");
    const uint64_t bytes = (uint64_t)a.n * a.n;
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(d_buf0), p1 = reinterpret_cast<uintptr_t>(d_buf1);
    if (p0 < p1 + bytes && p1 < p0 + bytes)
        return set_error(FRACTAL_E_INVAL, "the two buffers overlap");
    if (steps < 0)
        return set_error(FRACTAL_E_INVAL, "steps must be >= 0");
    uint8_t *bufs[2] = {static_cast<uint8_t *>(d_buf0), static_cast<uint8_t *>(d_buf1)};
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int t = 0; t < steps; ++t) {
        a.src = bufs[t & 1];
        a.dst = bufs[(t + 1) & 1];
        if ((rc = nbb_launch<NBB_CA>(map, a, s)))
            return rc;
    }
    return FRACTAL_OK;
}

} // extern "C"
