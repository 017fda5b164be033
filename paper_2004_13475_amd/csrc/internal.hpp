// internal.hpp -- host-side declarations shared by the library's translation
// units (launchers, error reporting, tuning).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fractal.h"

namespace fractal {

enum : int { MAP_LAMBDA = 0, MAP_BB = 1, MAP_MFMA = 2 };

constexpr int kMaxStepLevel = 16; // k for step calls (64-bit offsets inside)
constexpr int kMaxBlockLevel = 15; // k - r for step calls (grid limits)
constexpr int kMaxR = 6;           // rho <= 64
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator dies, 32 CUs each

// Error reporting (thread-local message).
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_error(hipError_t e, const char *what);

inline size_t cell_bytes(int rule) { return rule == FRACTAL_RULE_CA ? 1u : 4u; }
inline size_t state_bytes(int k, int rule)
{
    return ((size_t)1 << (2 * k)) * cell_bytes(rule);
}
inline uint64_t pow3_u64(int e)
{
    uint64_t p = 1;
    for (int i = 0; i < e; ++i)
        p *= 3;
    return p;
}

// Host-side checks shared by every step entry point.
int check_step_args(int k, int r, int rule, float alpha, const void *b0,
                    const void *b1, int steps);
int check_tuning(int map, int k, int rule, const fractal_tuning *t);

// Default / cached tuning for a lambda launch of (k, rule).
fractal_tuning default_tuning(int k, int rule);
fractal_tuning tuning_for_r(int map, int k, int rule, int r);

// Launch `steps` step kernels (validated arguments).
int launch_steps(int map, int k, int rule, float alpha, void *b0, void *b1,
                 int steps, const fractal_tuning &t, hipStream_t s);

// lambda map kernels.
int launch_lambda_map(int k, int r, uint32_t *d_xy, bool mfma, hipStream_t s);

// Seeded state fill.
int launch_seed_fill(int k, int rule, uint32_t stream_id, void *d_buf,
                     hipStream_t s);

// Sum of a state's cell bit patterns into *d_out (device uint64), added.
int launch_checksum(int k, int rule, const void *d_buf,
                    unsigned long long *d_out, hipStream_t s);

// Batched persistent step: device table entry per instance.
struct BatchEntry {
    uint64_t tile_begin; // prefix of 3^(k_j - r_j) over earlier entries
    uint8_t *buf0;
    uint8_t *buf1;
    int32_t k;
    int32_t r;
    int32_t rule;
    int32_t phase; // steps already done by this instance (parity source)
    float alpha;
    int32_t pad;
};
static_assert(sizeof(BatchEntry) == 48, "BatchEntry layout");

// One batched launch over the first `count` table entries (sorted so that the
// active ones form a prefix): tiles [0, total_tiles) of step `local_step`.
int launch_batch(const BatchEntry *d_table, int count, uint64_t total_tiles,
                 int local_step, int grid, hipStream_t s);
int batch_supported_r(int rule, int r);
int batch_default_r(int k, int rule);
int batch_grid_size();

} // namespace fractal
