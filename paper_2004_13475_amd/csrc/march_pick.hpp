// march_pick.hpp -- instantiation of the register-march step kernels for
// one rule (each rule's kernels are compiled in a source of their own).
#pragma once

#include <hip/hip_runtime.h>

#include "device_march.hpp"
#include "internal.hpp"

namespace fractal {

// The kernel for a launch shape; ALT selects the other occupancy where
// the lambda map has a kernel for it (march_has_alt), else the default one.
template <int MAP, int RULE, int R, int T, int FL, bool ALT>
static MarchFn march_fn()
{
    constexpr int HL = march_hl(RULE, T);
    if constexpr (MGeom<RULE, R, T, HL>::VALID && march_supported(RULE, T, R)) {
        if constexpr (ALT && MAP == MAP_LAMBDA && march_has_alt(RULE, T, R))
            return march_kernel<RULE, R, T, HL, MAP, FL, march_wpe_alt(T), march_depth(RULE, T)>;
        else
            return march_kernel<RULE, R, T, HL, MAP, FL, march_wpe(T), march_depth(RULE, T)>;
    } else {
        return nullptr;
    }
}

template <int MAP, int RULE, int FL, bool ALT>
static MarchFn march_pick_rt(int r, int T)
{
    switch (r) {
#define FRACTAL_MARCH_R(RR)                                                                        \
    case RR:                                                                                       \
        switch (T) {                                                                               \
        case 1: return march_fn<MAP, RULE, RR, 1, FL, false>();                                    \
        case 2: return march_fn<MAP, RULE, RR, 2, FL, false>();                                    \
        case 4: return march_fn<MAP, RULE, RR, 4, FL, false>();                                    \
        case 8: return march_fn<MAP, RULE, RR, 8, FL, ALT>();                                      \
        case 16: return march_fn<MAP, RULE, RR, 16, FL, ALT>();                                    \
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

template <int RULE>
static MarchFn march_pick_rule(int map, int r, int T, bool nt, bool alt)
{
    if (map == MAP_LAMBDA && alt)
        return nt ? march_pick_rt<MAP_LAMBDA, RULE, TILE_NT_STORE, true>(r, T)
                  : march_pick_rt<MAP_LAMBDA, RULE, 0, true>(r, T);
    if (map == MAP_LAMBDA)
        return nt ? march_pick_rt<MAP_LAMBDA, RULE, TILE_NT_STORE, false>(r, T)
                  : march_pick_rt<MAP_LAMBDA, RULE, 0, false>(r, T);
    if (map == MAP_BB)
        return nt ? march_pick_rt<MAP_BB, RULE, TILE_NT_STORE, false>(r, T)
                  : march_pick_rt<MAP_BB, RULE, 0, false>(r, T);
    return nullptr;
}

// Lambda-map kernels of 10 and 12 steps per launch, tiles of side 16, 32
// and 64: the launch sizes between 8 and 16 that let a call of a
// sixteen-step tuning split its steps evenly.
template <int RULE, int FL>
static MarchFn march_pick_mid_r(int r, int T)
{
    switch (r) {
#define FRACTAL_MARCH_MID_R(RR)                                                                    \
    case RR:                                                                                       \
        switch (T) {                                                                               \
        case 10: return march_fn<MAP_LAMBDA, RULE, RR, 10, FL, false>();                           \
        case 12: return march_fn<MAP_LAMBDA, RULE, RR, 12, FL, false>();                           \
        default: return nullptr;                                                                   \
        }
        FRACTAL_MARCH_MID_R(4)
        FRACTAL_MARCH_MID_R(5)
        FRACTAL_MARCH_MID_R(6)
#undef FRACTAL_MARCH_MID_R
    default: return nullptr;
    }
}

template <int RULE>
static MarchFn march_pick_mid_rule(int r, int T, bool nt)
{
    return nt ? march_pick_mid_r<RULE, TILE_NT_STORE>(r, T) : march_pick_mid_r<RULE, 0>(r, T);
}

} // namespace fractal
