// device_map.hpp -- block-space maps for gfx950: lambda(omega) per wavefront
// (Theorem 1, Section 6.1), its matrix-core form (Section 6.3, Variant 1),
// and the dispatch orders that turn a hardware workgroup id into omega.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fractal.h"

namespace fractal {

struct TileXY {
    uint32_t x, y; // block (tile) coordinates in the n_b x n_b block space
};

// 3^e modulo 2^32 for 0 <= e < 32 (exact while e <= 20).
__device__ __forceinline__ uint32_t pow3_u32(uint32_t e)
{
    uint32_t p = 1u, b = 3u;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (e & (1u << i))
            p *= b;
        b *= b;
    }
    return p;
}

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// The gasket's replica table maps beta = 0, 1, 2 to offsets (0,0), (0,1),
// (1,1) in the paper's orientation.  Each level's offset is tau * 2^(mu-1),
// so the levels fill disjoint bits and the sum over levels is a bit pattern:
// bit mu-1 of lambda_x is [beta_mu == 2]; bit mu-1 of the paper's lambda_y is
// [beta_mu != 0], which after the vertical mirror (n_b - 1 - lambda_y) is
// [beta_mu == 0].  Lane j holds beta_{j+1}; two ballots assemble both
// coordinates in scalar registers, uniform across the wavefront.
// Must be called by all 64 lanes of the wavefront.
__device__ __forceinline__ TileXY ballot_assemble(uint32_t beta, int rb)
{
    const bool act = lane_id() < (uint32_t)rb;
    const uint64_t bx = __builtin_amdgcn_ballot_w64(act && beta == 2u);
    const uint64_t by = __builtin_amdgcn_ballot_w64(act && beta == 0u);
    return TileXY{(uint32_t)bx, (uint32_t)by};
}

// beta_mu(omega) = floor(v / 3^(ceil(mu/2)-1)) mod 3 with v = omega_x for odd
// mu and omega_y for even mu (the selector of the helper's formula), computed
// for mu = lane + 1.
__device__ __forceinline__ uint32_t beta_of_omega(uint32_t wx, uint32_t wy,
                                                  uint32_t mu)
{
    const uint32_t v = (mu & 1u) ? wx : wy;
    const uint32_t q = v / pow3_u32((mu + 1u) / 2u - 1u);
    return q - 3u * (q / 3u);
}

// lambda(omega) for omega in the 3^ceil(rb/2) x 3^floor(rb/2) grid.
__device__ __forceinline__ TileXY lambda_wave(uint32_t wx, uint32_t wy, int rb)
{
    return ballot_assemble(beta_of_omega(wx, wy, lane_id() + 1u), rb);
}

// Linear id L whose base-3 digit mu-1 is beta_mu: the omega with
// omega_x = digits at odd mu and omega_y = digits at even mu.  Consecutive L
// walk the gasket's self-similar order, so consecutive workgroups touch
// neighbouring tiles.
__device__ __forceinline__ TileXY lambda_wave_curve(uint32_t L, int rb)
{
    const uint32_t q = L / pow3_u32(lane_id());
    return ballot_assemble(q - 3u * (q / 3u), rb);
}

// lambda for one tile per lane, as the register-march kernels evaluate it
// (their wavefronts hold several tiles, so each lane group needs its own
// lambda): block coordinates of tile `id`, where base-3 digit mu-1 of the id
// (CURVE orders) or of omega_x / omega_y for odd / even mu (NATURAL,
// omega = (id mod gx, id div gx)) is beta_mu; bit mu-1 of x is [beta == 2]
// and of y is [beta == 0] (the mirrored replica table).  rb <= 20.
__device__ __forceinline__ TileXY lambda_lane(uint32_t id, int rb, int order)
{
    uint32_t a = id, b = 0u;
    if (order == FRACTAL_ORDER_NATURAL) {
        const uint32_t gx = pow3_u32((uint32_t)(rb + 1) / 2u);
        b = id / gx;
        a = id - b * gx;
    }
    uint32_t x = 0u, y = 0u;
    for (int mu = 0; mu < rb; ++mu) {
        uint32_t d;
        if (order == FRACTAL_ORDER_NATURAL && (mu & 1)) {
            const uint32_t q = b / 3u;
            d = b - 3u * q;
            b = q;
        } else {
            const uint32_t q = a / 3u;
            d = a - 3u * q;
            a = q;
        }
        x |= (uint32_t)(d == 2u) << mu;
        y |= (uint32_t)(d == 0u) << mu;
    }
    return TileXY{x, y};
}

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Section 6.3, Variant 1 on a 16x16x16 float16 matrix-core product:
// A row 0 = (2^0, ..., 2^(rb-1), 0, ...), B column 0 = tau_x^mu,
// column 1 = tau_y^mu (row mu-1), everything else 0; D[0][0] and D[0][1] are
// the sums of Eqs. lambda-x and lambda-y (paper orientation).  Every operand
// is an integer below 2^16 and every partial sum below 2^16, so float16
// inputs and float32 accumulation are exact.  Operand layout of
// v_mfma_f32_16x16x16_f16: lane l holds A[l%16][4*(l/16)+t] and
// B[4*(l/16)+t][l%16] for t = 0..3, and D[4*(l/16)+t][l%16].
// `beta_for` returns beta_mu for a level mu (1-based).  Requires rb <= 16.
template <class BetaFn>
__device__ __forceinline__ TileXY lambda_mfma(BetaFn beta_for, int rb)
{
    const uint32_t l = lane_id();
    const uint32_t row = l & 15u, kb = 4u * (l >> 4);
    half4_t a, b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const uint32_t kk = kb + (uint32_t)t; // contraction index = mu - 1
        const bool live = kk < (uint32_t)rb;
        // A: only row 0 is non-zero
        a[t] = (row == 0u && live) ? (_Float16)(float)(1u << kk) : (_Float16)0.0f;
        // B: column 0 = tau_x = [beta == 2], column 1 = tau_y = [beta != 0]
        uint32_t beta = live ? beta_for(kk + 1u) : 0u;
        float tau = 0.0f;
        if (row == 0u)
            tau = (beta == 2u) ? 1.0f : 0.0f;
        else if (row == 1u)
            tau = (beta != 0u) ? 1.0f : 0.0f;
        b[t] = (_Float16)tau;
    }
    float4_t c = {0.0f, 0.0f, 0.0f, 0.0f};
    float4_t d = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    // D[0][0] in lane 0 element 0, D[0][1] in lane 1 element 0
    const uint32_t px = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)d[0], 0);
    const uint32_t py = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)d[0], 1);
    const uint32_t nb1 = (1u << rb) - 1u;
    return TileXY{px, nb1 - py};
}

// lambda^-1: the curve index of non-empty tile (x, y) of a level-rb tile
// space, the inverse of lambda on the curve order: base-3 digit mu-1 is 2
// where bit mu-1 of x is set, 0 where that of y is set, 1 where neither.
__device__ __forceinline__ uint32_t lambda_inverse(uint32_t x, uint32_t y, int rb)
{
    uint32_t L = 0u;
    for (int mu = rb - 1; mu >= 0; --mu) {
        const uint32_t bx = (x >> mu) & 1u, by = (y >> mu) & 1u;
        L = 3u * L + (bx ? 2u : (by ? 0u : 1u));
    }
    return L;
}

// Split [0, N) into 8 contiguous ranges, one per accelerator die: hardware
// workgroup b runs on die b % 8 (round-robin dispatch), and becomes the
// (b / 8)-th id of that die's range.  A bijection of [0, N).
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t b, uint32_t N)
{
    const uint32_t x = b & 7u, i = b >> 3;
    const uint32_t q = N >> 3, rem = N & 7u;
    return x * q + (x < rem ? x : rem) + i;
}

} // namespace fractal
