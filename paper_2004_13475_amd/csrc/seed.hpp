// seed.hpp -- the seeded cell value (input plumbing; no part of the map or
// the stencils), shared by the embedded and compact seed fills.
//
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): cell (x, y) of stream id
// s draws output number i+1 of a SplitMix64 started from state 0,
// i = s * 2^32 + y * n + x (mod 2^64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fractal.h"

namespace fractal {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t i)
{
    uint64_t z = (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Cell value as a 32-bit pattern: automaton top bit, heat (z >> 40) * 2^-24;
// 0 off the gasket.
template <int RULE>
__device__ __forceinline__ uint32_t seeded_cell(uint64_t base, uint32_t x, uint32_t y, int k)
{
    if ((x & y) != 0u)
        return 0u;
    const uint64_t z = splitmix64_at(base + ((uint64_t)y << k) + x);
    if constexpr (RULE == FRACTAL_RULE_CA)
        return (uint32_t)(z >> 63);
    else
        return __float_as_uint((float)(uint32_t)(z >> 40) * 0x1.0p-24f);
}

} // namespace fractal
