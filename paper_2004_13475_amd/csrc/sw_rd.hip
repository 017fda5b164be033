// sw_rd.hip -- tests SW (single write) and RD (reduction) of the paper's
// case study (Section 6.2) on the lambda and bounding-box maps.
//
// A wavefront takes P tiles side by side; a tile's lanes each own one
// chunk column (16 bytes, or the whole row of a narrower tile) and walk the
// tile's rows.  SW writes every 64-byte segment that holds a member (value on
// members, 0 elsewhere in the segment); RD loads every chunk that holds a
// member and sums its members, lanes of a tile combine their sums by a fixed
// butterfly, and the tile's sum goes to slot lambda^-1(tile) of the
// workspace; a fixed summation tree then reduces the slots.  Nothing depends
// on which map dispatched a tile or when, so lambda and BB agree bit for bit.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_map.hpp"
#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

template <int RULE, int R>
struct SGeom {
    static constexpr int S = (RULE == RULE_CA) ? 1 : 4;
    static constexpr int RHO = 1 << R;
    static constexpr int RB = RHO * S;               // tile row bytes
    static constexpr int CB = RB < 16 ? RB : 16;     // bytes per lane chunk
    static constexpr int CC = CB / S;                // cells per chunk
    static constexpr int IL = RB / CB;               // lanes per tile (power of two)
    static constexpr int P = 64 / IL;                // tiles per wavefront
    static constexpr int SLOG = (RULE == RULE_CA) ? 6 : 4; // cells per 64-byte segment (log2)
};

struct SwRdArgs {
    uint8_t *buf;
    int k;
    int rb;
    uint64_t total;   // tiles in the map's id space
    uint32_t value;   // SW
    uint64_t *slots;  // RD: one 8-byte partial per non-empty tile
};

template <int CB>
__device__ __forceinline__ void chunk_load(const uint8_t *p, uint8_t (&b)[CB])
{
    if constexpr (CB == 16) {
        const u32x4 v = *reinterpret_cast<const u32x4 *>(p);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            b[i] = (uint8_t)(v[i >> 2] >> (8 * (i & 3)));
    } else if constexpr (CB == 8) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            b[i] = (uint8_t)(((i < 4) ? v.x : v.y) >> (8 * (i & 3)));
    } else if constexpr (CB == 4) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            b[i] = (uint8_t)(v >> (8 * i));
    } else {
#pragma unroll
        for (int i = 0; i < CB; ++i)
            b[i] = p[i];
    }
}

template <int CB>
__device__ __forceinline__ void chunk_store(uint8_t *p, const uint8_t (&b)[CB])
{
    if constexpr (CB >= 4) {
        uint32_t w[CB / 4];
#pragma unroll
        for (int q = 0; q < CB / 4; ++q)
            w[q] = (uint32_t)b[4 * q] | ((uint32_t)b[4 * q + 1] << 8) |
                   ((uint32_t)b[4 * q + 2] << 16) | ((uint32_t)b[4 * q + 3] << 24);
        if constexpr (CB == 16)
            *reinterpret_cast<u32x4 *>(p) = u32x4{w[0], w[1], w[2], w[3]};
        else if constexpr (CB == 8)
            *reinterpret_cast<uint2 *>(p) = uint2{w[0], w[1]};
        else
            *reinterpret_cast<uint32_t *>(p) = w[0];
    } else {
#pragma unroll
        for (int i = 0; i < CB; ++i)
            p[i] = b[i];
    }
}

// Sum of v over the IL lanes of this lane's group (aligned runs of IL lanes),
// by a fixed butterfly; every lane of the group ends with the same bits.
template <int IL>
__device__ __forceinline__ uint64_t group_sum_u64(uint64_t v)
{
#pragma unroll
    for (int off = 1; off < IL; off <<= 1) {
        const int src = (int)((lane_id() ^ (uint32_t)off) << 2);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)v);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(v >> 32));
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

template <int IL>
__device__ __forceinline__ double group_sum_f64(double v)
{
#pragma unroll
    for (int off = 1; off < IL; off <<= 1) {
        const int src = (int)((lane_id() ^ (uint32_t)off) << 2);
        const uint64_t bits = (uint64_t)__double_as_longlong(v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)bits);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(bits >> 32));
        const double o = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
        // a + b and b + a are the same float64, so both partners agree
        v = (lane_id() & (uint32_t)off) ? o + v : v + o;
    }
    return v;
}

enum : int { OP_SW = 0, OP_RD = 1 };

template <int RULE, int R, int MAP, int OP>
__global__ __launch_bounds__(256) void swrd_kernel(SwRdArgs a)
{
    using G = SGeom<RULE, R>;
    const uint32_t lane = lane_id();
    const uint32_t grp = lane / (uint32_t)G::IL;
    const int col = (int)(lane - grp * (uint32_t)G::IL);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t tile = wave * G::P + grp;
    bool active = tile < a.total;
    uint32_t tx = 0u, ty = 0u, slot = 0u;
    if (active) {
        if constexpr (MAP == MAP_BB) {
            tx = (uint32_t)tile & ((1u << a.rb) - 1u);
            ty = (uint32_t)(tile >> a.rb);
            active = (tx & ty) == 0u;
            if (active)
                slot = lambda_inverse(tx, ty, a.rb);
        } else {
            const TileXY t = lambda_lane((uint32_t)tile, a.rb, FRACTAL_ORDER_CURVE);
            tx = t.x;
            ty = t.y;
            slot = (uint32_t)tile;
        }
    }
    if constexpr (OP == OP_SW) {
        if (!active)
            return;
    } else {
        if (__builtin_amdgcn_ballot_w64(active) == 0u)
            return; // the group sums below need every lane of the wavefront
    }
    const uint32_t n = 1u << a.k;
    const uint32_t x = (tx << R) + (uint32_t)col * G::CC;
    const uint32_t y0 = ty << R;
    uint8_t *base = a.buf + ((uint64_t)y0 * n + x) * G::S;
    const uint64_t pitch = (uint64_t)n * G::S;
    uint32_t acc_u = 0u;
    double acc_d = 0.0;
    if constexpr (OP == OP_RD && G::CB == 16) {
        // rows in groups of UR: every lane issues the group's loads before
        // it adds (a chunk without a member reads the buffer's first chunk,
        // always valid, and is skipped), so UR loads are in flight at once
        constexpr int UR = G::RHO < 8 ? G::RHO : 8;
        using gu32x4 = const __attribute__((address_space(1))) u32x4;
        for (int j0 = 0; j0 < G::RHO; j0 += UR) {
            u32x4 v[UR];
            bool has[UR];
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const uint32_t y = y0 + (uint32_t)(j0 + u);
                has[u] = active && (x & y) == 0u;
                v[u] = *(gu32x4 *)(has[u] ? base + (uint64_t)(j0 + u) * pitch : a.buf);
            }
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                if (!has[u])
                    continue;
                const uint32_t y = y0 + (uint32_t)(j0 + u);
#pragma unroll
                for (int c = 0; c < G::CC; ++c) {
                    const bool m = (((uint32_t)c) & y) == 0u;
                    if constexpr (RULE == RULE_CA)
                        acc_u += m ? ((v[u][c >> 2] >> (8 * (c & 3))) & 0xFFu) : 0u;
                    else
                        acc_d += m ? (double)__uint_as_float(v[u][c]) : 0.0;
                }
            }
        }
    } else
    for (int j = 0; j < G::RHO; ++j) {
        const uint32_t y = y0 + (uint32_t)j;
        uint8_t *p = base + (uint64_t)j * pitch;
        if constexpr (OP == OP_SW) {
            if (((x >> G::SLOG) & (y >> G::SLOG)) != 0u)
                continue; // no member in this 64-byte segment
            uint8_t b[G::CB];
#pragma unroll
            for (int c = 0; c < G::CC; ++c) {
                const bool m = ((x + (uint32_t)c) & y) == 0u;
#pragma unroll
                for (int q = 0; q < G::S; ++q)
                    b[c * G::S + q] = m ? (uint8_t)(a.value >> (8 * q)) : (uint8_t)0;
            }
            chunk_store<G::CB>(p, b);
        } else {
            if (!active || (x & y) != 0u)
                continue; // no member in this chunk
            uint8_t b[G::CB];
            chunk_load<G::CB>(p, b);
#pragma unroll
            for (int c = 0; c < G::CC; ++c) {
                const bool m = (((uint32_t)c) & y) == 0u;
                if constexpr (RULE == RULE_CA) {
                    acc_u += m ? b[c] : 0u;
                } else {
                    const uint32_t bits = (uint32_t)b[4 * c] | ((uint32_t)b[4 * c + 1] << 8) |
                                          ((uint32_t)b[4 * c + 2] << 16) |
                                          ((uint32_t)b[4 * c + 3] << 24);
                    acc_d += m ? (double)__uint_as_float(bits) : 0.0;
                }
            }
        }
    }
    if constexpr (OP == OP_RD) {
        uint64_t out;
        if constexpr (RULE == RULE_CA)
            out = group_sum_u64<G::IL>((uint64_t)acc_u);
        else
            out = (uint64_t)__double_as_longlong(group_sum_f64<G::IL>(acc_d));
        if (active && col == 0)
            a.slots[slot] = out;
    }
}

// One pass of the summation tree: workgroup b sums in[b*4096 .. +4096) --
// thread t adds elements t, t + 256, ... in order, then a fixed LDS tree.
template <bool F64>
__global__ __launch_bounds__(256) void tree_kernel(const uint64_t *__restrict__ in, uint64_t n,
                                                   uint64_t *__restrict__ out)
{
    __shared__ uint64_t sh[256];
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * 4096u + t;
    uint64_t acc_u = 0u;
    double acc_d = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint64_t e = base + 256u * (uint64_t)i;
        if (e < n) {
            if constexpr (F64)
                acc_d += __longlong_as_double((long long)in[e]);
            else
                acc_u += in[e];
        }
    }
    sh[t] = F64 ? (uint64_t)__double_as_longlong(acc_d) : acc_u;
    __syncthreads();
    for (uint32_t s = 128; s > 0; s >>= 1) {
        if (t < s) {
            if constexpr (F64)
                sh[t] = (uint64_t)__double_as_longlong(__longlong_as_double((long long)sh[t]) +
                                                       __longlong_as_double((long long)sh[t + s]));
            else
                sh[t] += sh[t + s];
        }
        __syncthreads();
    }
    if (t == 0)
        out[blockIdx.x] = sh[0];
}

typedef void (*SwRdFn)(SwRdArgs);

template <int RULE, int MAP, int OP>
static SwRdFn swrd_pick_r(int r)
{
    switch (r) {
    case 0: return swrd_kernel<RULE, 0, MAP, OP>;
    case 1: return swrd_kernel<RULE, 1, MAP, OP>;
    case 2: return swrd_kernel<RULE, 2, MAP, OP>;
    case 3: return swrd_kernel<RULE, 3, MAP, OP>;
    case 4: return swrd_kernel<RULE, 4, MAP, OP>;
    case 5: return swrd_kernel<RULE, 5, MAP, OP>;
    case 6: return swrd_kernel<RULE, 6, MAP, OP>;
    case 7: return swrd_kernel<RULE, 7, MAP, OP>;
    default: return nullptr;
    }
}

template <int OP>
static SwRdFn swrd_pick(int map, int rule, int r)
{
    if (map == MAP_BB)
        return rule == FRACTAL_RULE_CA ? swrd_pick_r<RULE_CA, MAP_BB, OP>(r)
                                       : swrd_pick_r<RULE_HEAT, MAP_BB, OP>(r);
    return rule == FRACTAL_RULE_CA ? swrd_pick_r<RULE_CA, MAP_LAMBDA, OP>(r)
                                   : swrd_pick_r<RULE_HEAT, MAP_LAMBDA, OP>(r);
}

static int tiles_per_wave(int rule, int r)
{
    const int rbytes = (1 << r) * (int)cell_bytes(rule);
    const int cb = rbytes < 16 ? rbytes : 16;
    return 64 / (rbytes / cb);
}

static int check_swrd(int map, int k, int r, int rule, const void *buf)
{
    if (map != MAP_LAMBDA && map != MAP_BB)
        return set_error(FRACTAL_E_INVAL, "map %d: SW and RD run on lambda (0) or BB (1)", map);
    if (k < 0 || k > kMaxStepLevel || r < 0 || r > k || r > kMaxR || k - r > kMaxBlockLevel)
        return set_error(FRACTAL_E_INVAL, "need 0 <= r <= min(k, %d), k <= %d, k - r <= %d "
                         "(k=%d r=%d)", kMaxR, kMaxStepLevel, kMaxBlockLevel, k, r);
    if (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT)
        return set_error(FRACTAL_E_INVAL, "unknown rule %d", rule);
    if (!buf)
        return set_error(FRACTAL_E_INVAL, "null buffer");
    if (reinterpret_cast<uintptr_t>(buf) % 16)
        return set_error(FRACTAL_E_INVAL, "buffer must be 16-byte aligned");
    return FRACTAL_OK;
}

static int launch_swrd(SwRdFn fn, int rule, int r, const SwRdArgs &a, hipStream_t s)
{
    const uint64_t P = (uint64_t)tiles_per_wave(rule, r);
    const uint64_t waves = (a.total + P - 1) / P;
    const uint64_t grid = (waves + 3) / 4;
    SwRdArgs arg = a;
    void *args[] = {&arg};
    return hip_error(hipLaunchKernel((const void *)fn, dim3((unsigned)grid), dim3(256), args, 0, s),
                     "SW/RD kernel launch");
}

// Sizes of the summation tree's levels: n_0 slots, then ceil(n_i / 4096)
// until one value remains (that one is the result).  A fixed-size record:
// 4096-ary levels over at most 3^15 slots take four sizes.
struct TreeLevels {
    uint64_t n[8];
    int count;
};

static TreeLevels tree_levels(uint64_t n0)
{
    TreeLevels lv{};
    lv.n[0] = n0;
    lv.count = 1;
    while (lv.n[lv.count - 1] > 1 && lv.count < 8) {
        lv.n[lv.count] = (lv.n[lv.count - 1] + 4095) / 4096;
        ++lv.count;
    }
    if (lv.count == 1)
        lv.n[lv.count++] = 1; // one slot still takes one pass
    return lv;
}

uint64_t reduce_tree_words(uint64_t n0)
{
    const TreeLevels lv = tree_levels(n0);
    uint64_t words = 0;
    for (int i = 0; i + 1 < lv.count; ++i)
        words += lv.n[i];
    return words;
}

int launch_reduce_tree(uint64_t *work, uint64_t n0, void *d_out, bool f64, hipStream_t s)
{
    const TreeLevels lv = tree_levels(n0);
    uint64_t *in = work;
    for (int i = 0; i + 1 < lv.count; ++i) {
        uint64_t *out = (i + 2 == lv.count) ? static_cast<uint64_t *>(d_out) : in + lv.n[i];
        if (f64)
            hipLaunchKernelGGL(tree_kernel<true>, dim3((unsigned)lv.n[i + 1]), dim3(256), 0, s, in,
                               lv.n[i], out);
        else
            hipLaunchKernelGGL(tree_kernel<false>, dim3((unsigned)lv.n[i + 1]), dim3(256), 0, s, in,
                               lv.n[i], out);
        int rc = hip_error(hipGetLastError(), "reduction tree launch");
        if (rc)
            return rc;
        in = out;
    }
    return FRACTAL_OK;
}

// Workspace of fractal_reduce_noalloc: one per device, allocated with the
// code object and held until the process ends.  Host code never uses this
// name as an address (on the host it is only a stand-in for the symbol):
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) uint64_t scratch[kNoallocScratchBytes / 8];

constexpr int kNoallocMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t *g_scratch_ptr[kNoallocMaxDevices];

// The calling thread's current device's copy of `scratch`, looked up on the
// first call on that device.
static int noalloc_scratch(uint64_t **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoallocMaxDevices)
        return set_error(FRACTAL_E_DEVICE, "device %d beyond the %d devices the scratch table holds",
                         dev, kNoallocMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return set_error(FRACTAL_E_DEVICE, "scratch has no device address");
        g_scratch_ptr[dev] = static_cast<uint64_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return FRACTAL_OK;
}

} // namespace fractal

using namespace fractal;

extern "C" {

int fractal_single_write(int map, int k, int r, int rule, uint32_t value, void *d_buf,
                         void *stream)
{
    int rc = check_swrd(map, k, r, rule, d_buf);
    if (rc)
        return rc;
    SwRdArgs a;
    a.buf = static_cast<uint8_t *>(d_buf);
    a.k = k;
    a.rb = k - r;
    a.total = map == MAP_BB ? (uint64_t)1 << (2 * (k - r)) : pow3_u64(k - r);
    a.value = value;
    a.slots = nullptr;
    return launch_swrd(swrd_pick<OP_SW>(map, rule, r), rule, r, a, static_cast<hipStream_t>(stream));
}

int fractal_reduce_workspace(int k, int r, size_t *bytes)
{
    if (!bytes)
        return set_error(FRACTAL_E_INVAL, "null output");
    if (k < 0 || k > kMaxStepLevel || r < 0 || r > k || r > kMaxR || k - r > kMaxBlockLevel)
        return set_error(FRACTAL_E_INVAL, "bad level k=%d r=%d", k, r);
    const uint64_t words = reduce_tree_words(pow3_u64(k - r));
    *bytes = (size_t)(8 * words);
    return FRACTAL_OK;
}

int fractal_reduce(int map, int k, int r, int rule, const void *d_buf, void *d_work,
                   size_t work_bytes, void *d_out, void *stream)
{
    int rc = check_swrd(map, k, r, rule, d_buf);
    if (rc)
        return rc;
    size_t need = 0;
    if ((rc = fractal_reduce_workspace(k, r, &need)))
        return rc;
    if (!d_work || !d_out)
        return set_error(FRACTAL_E_INVAL, "null workspace or output");
    if (reinterpret_cast<uintptr_t>(d_work) % 8 || reinterpret_cast<uintptr_t>(d_out) % 8)
        return set_error(FRACTAL_E_INVAL, "workspace and output must be 8-byte aligned");
    if (work_bytes < need)
        return set_error(FRACTAL_E_INVAL, "workspace of %zu bytes, %zu needed", work_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t *w = static_cast<uint64_t *>(d_work);
    SwRdArgs a;
    a.buf = static_cast<uint8_t *>(const_cast<void *>(d_buf));
    a.k = k;
    a.rb = k - r;
    a.total = map == MAP_BB ? (uint64_t)1 << (2 * (k - r)) : pow3_u64(k - r);
    a.value = 0;
    a.slots = w;
    if ((rc = launch_swrd(swrd_pick<OP_RD>(map, rule, r), rule, r, a, s)))
        return rc;
    if ((rc = launch_reduce_tree(w, pow3_u64(k - r), d_out, rule == FRACTAL_RULE_HEAT, s)))
        return rc;
    return FRACTAL_OK;
}

int fractal_reduce_noalloc(int map, int k, int r, int rule, const void *d_buf, void *d_out,
                           void *stream)
{
    int rc = check_swrd(map, k, r, rule, d_buf);
    if (rc)
        return rc;
    size_t need = 0;
    if ((rc = fractal_reduce_workspace(k, r, &need)))
        return rc;
    if (need > kNoallocScratchBytes)
        return set_error(FRACTAL_E_INVAL,
                         "k=%d r=%d needs %zu bytes of scratch, the static scratch holds %zu "
                         "(k - r <= 13); use fractal_reduce with a workspace",
                         k, r, need, kNoallocScratchBytes);
    if (!d_out || reinterpret_cast<uintptr_t>(d_out) % 8)
        return set_error(FRACTAL_E_INVAL, "output must be non-null and 8-byte aligned");
    uint64_t *w = nullptr;
    if ((rc = noalloc_scratch(&w)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SwRdArgs a;
    a.buf = static_cast<uint8_t *>(const_cast<void *>(d_buf));
    a.k = k;
    a.rb = k - r;
    a.total = map == MAP_BB ? (uint64_t)1 << (2 * (k - r)) : pow3_u64(k - r);
    a.value = 0;
    a.slots = w;
    // every slot is written by the tile it belongs to before the tree reads
    // it, so the scratch needs no clearing between calls
    if ((rc = launch_swrd(swrd_pick<OP_RD>(map, rule, r), rule, r, a, s)))
        return rc;
    return launch_reduce_tree(w, pow3_u64(k - r), d_out, rule == FRACTAL_RULE_HEAT, s);
}

} // extern "C"
