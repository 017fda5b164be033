// internal.hpp -- host-side declarations shared by the library's translation
// units (launchers, error reporting, tuning).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

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

// Batched steps: device table entry per instance.
struct BatchEntry {
    uint64_t tile_begin; // prefix of 3^(k_j - r) over earlier entries of the class
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

// One gasket advanced by a batched launch sequence.
struct BatchItem {
    int k, rule;
    int steps; // steps to run in this sequence (local steps 0..steps-1)
    int phase; // steps done before (input is buf[phase & 1])
    float alpha;
    uint8_t *buf0, *buf1;
    fractal_tuning tuning; // tile launch (r, threads, flags) for this item
};

// Instances grouped by launch class (rule, r, threads, step flags); each
// class is a contiguous run of table entries sorted by steps (descending),
// so the items still running at local step j form a prefix of the class.
class BatchPlan {
  public:
    // Fills `host` (capacity >= items.size()) and records the classes.
    void build(const std::vector<BatchItem> &items, BatchEntry *host);
    // Launch local step j of every class whose prefix is non-empty.
    int launch_step(const BatchEntry *d_table, int j, bool persistent, hipStream_t s) const;
    int max_steps() const { return max_steps_; }
    size_t entries() const { return entries_; }

  private:
    struct Class {
        int rule, r, threads, flags;
        size_t first;
        std::vector<int> steps;       // per entry, descending
        std::vector<uint64_t> prefix; // tile prefix, size steps.size() + 1
    };
    std::vector<Class> classes_;
    int max_steps_ = 0;
    size_t entries_ = 0;
};

// Tile launch used for one batched instance: `forced` (may be NULL) overrides
// the per-level cached or default tuning.
fractal_tuning batch_item_tuning(int k, int rule, const fractal_tuning *forced);

} // namespace fractal
