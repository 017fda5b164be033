// seed.hip -- seeded initial states and state checksums (input plumbing; no
// part of the map or the stencils).
//
// The seeded state follows SplitMix64 (Steele, Lea and Flood, OOPSLA 2014):
// cell (x, y) of stream id s draws output number i+1 of a SplitMix64 started
// from state 0, i = s * 2^32 + y * n + x.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "seed.hpp"

namespace fractal {

// Each thread fills one 16-byte chunk (16 automaton cells or 4 heat cells)
// of a row; rows narrower than a chunk are filled cell by cell.
template <int RULE>
__global__ __launch_bounds__(256) void seed_kernel(uint8_t *buf, int k, uint64_t base)
{
    constexpr int S = RULE == FRACTAL_RULE_CA ? 1 : 4;
    constexpr int CELLS = 16 / S;
    const uint32_t n = 1u << k;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < (uint32_t)CELLS) {
        const uint64_t cells = (uint64_t)n * n;
        for (uint64_t c = tid; c < cells; c += stride) {
            const uint32_t x = (uint32_t)(c & (n - 1)), y = (uint32_t)(c >> k);
            const uint32_t v = seeded_cell<RULE>(base, x, y, k);
            if constexpr (S == 1)
                buf[c] = (uint8_t)v;
            else
                reinterpret_cast<uint32_t *>(buf)[c] = v;
        }
        return;
    }
    const uint64_t chunks = ((uint64_t)n * n) / CELLS;
    for (uint64_t c = tid; c < chunks; c += stride) {
        const uint64_t cell0 = c * CELLS;
        const uint32_t x0 = (uint32_t)(cell0 & (n - 1)), y = (uint32_t)(cell0 >> k);
        uint32_t w[4];
        if constexpr (S == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t word = 0u;
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    word |= seeded_cell<RULE>(base, x0 + 4 * q + b, y, k) << (8 * b);
                w[q] = word;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                w[q] = seeded_cell<RULE>(base, x0 + q, y, k);
        }
        reinterpret_cast<uint4 *>(buf)[c] = uint4{w[0], w[1], w[2], w[3]};
    }
}

int launch_seed_fill(int k, int rule, uint32_t stream_id, void *d_buf, hipStream_t s)
{
    const uint64_t base = (uint64_t)stream_id << 32;
    const uint64_t work = ((uint64_t)1 << (2 * k)) / (rule == FRACTAL_RULE_CA ? 16 : 4) + 1;
    const uint64_t blocks = (work + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
    uint8_t *b = static_cast<uint8_t *>(d_buf);
    if (rule == FRACTAL_RULE_CA)
        hipLaunchKernelGGL(seed_kernel<FRACTAL_RULE_CA>, dim3(grid), dim3(256), 0, s, b, k, base);
    else
        hipLaunchKernelGGL(seed_kernel<FRACTAL_RULE_HEAT>, dim3(grid), dim3(256), 0, s, b, k, base);
    return hip_error(hipGetLastError(), "seed fill launch");
}

// Sum over all cells of the cell bit patterns (uint8 value or float32 bits)
// modulo 2^64, added into *out.  Each workgroup reduces its grid-stride share
// of 16-byte chunks and adds one partial with a single atomic.
template <int S>
__global__ __launch_bounds__(256) void checksum_kernel(const uint8_t *buf, uint64_t bytes,
                                                       unsigned long long *out)
{
    __shared__ unsigned long long part[256];
    unsigned long long acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t chunks = bytes / 16;
    for (uint64_t c = tid; c < chunks; c += stride) {
        const uint4 v = reinterpret_cast<const uint4 *>(buf)[c];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (S == 1)
                acc += (w[q] & 0xFFu) + ((w[q] >> 8) & 0xFFu) + ((w[q] >> 16) & 0xFFu) + (w[q] >> 24);
            else
                acc += w[q];
        }
    }
    for (uint64_t b = chunks * 16 + tid * S; b < bytes; b += stride * S) {
        if constexpr (S == 1)
            acc += buf[b];
        else
            acc += *reinterpret_cast<const uint32_t *>(buf + b);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicAdd(out, part[0]);
}

int launch_checksum(int k, int rule, const void *d_buf, unsigned long long *d_out,
                    hipStream_t s)
{
    const uint64_t bytes = state_bytes(k, rule);
    const uint64_t blocks = (bytes / 16 + 255) / 256 + 1;
    const unsigned grid = (unsigned)(blocks < 2048 ? blocks : 2048);
    const uint8_t *b = static_cast<const uint8_t *>(d_buf);
    if (rule == FRACTAL_RULE_CA)
        hipLaunchKernelGGL(checksum_kernel<1>, dim3(grid), dim3(256), 0, s, b, bytes, d_out);
    else
        hipLaunchKernelGGL(checksum_kernel<4>, dim3(grid), dim3(256), 0, s, b, bytes, d_out);
    return hip_error(hipGetLastError(), "checksum launch");
}

} // namespace fractal
