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
constexpr int kMaxR = 7;           // rho <= 128
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

// Arguments of one step-kernel launch.
struct StepLaunchArgs {
    const uint8_t *src; // state read by this launch
    uint8_t *dst;       // state written by this launch
    int k;              // level
    float alpha;        // heat coefficient
    int rb;             // block-space level k - r
    int order;          // FRACTAL_ORDER_*
    uint32_t total;     // workgroups in the grid
};
typedef void (*StepFn)(StepLaunchArgs);
StepFn pick_step(int map, int rule, int r, int threads, int flags);
StepFn pick_step_lambda(int rule, int r, int threads, int flags);
StepFn pick_step_bb(int rule, int r, int threads, int flags);
StepFn pick_step_mfma(int rule, int r, int threads, int flags);

// Steps one launch advances under these flags (1, 2, 4, 8, 16, or for the
// block engine 24, 32 or 36).
inline int launch_steps_of(int flags)
{
    return (flags & FRACTAL_FLAG_FUSE36)   ? 36
           : (flags & FRACTAL_FLAG_FUSE32) ? 32
           : (flags & FRACTAL_FLAG_FUSE24) ? 24
           : (flags & FRACTAL_FLAG_FUSE16) ? 16
           : (flags & FRACTAL_FLAG_FUSE8)  ? 8
           : (flags & FRACTAL_FLAG_FUSE4)  ? 4
           : (flags & FRACTAL_FLAG_FUSE2)  ? 2
                                           : 1;
}
constexpr int kDeepFlags = FRACTAL_FLAG_FUSE24 | FRACTAL_FLAG_FUSE32 | FRACTAL_FLAG_FUSE36; // block engine only
constexpr int kFuseFlags = FRACTAL_FLAG_FUSE2 | FRACTAL_FLAG_FUSE4 | FRACTAL_FLAG_FUSE8 |
                           FRACTAL_FLAG_FUSE16 | kDeepFlags;
constexpr int kStackFlags = FRACTAL_FLAG_STACK2 | FRACTAL_FLAG_STACK4 | FRACTAL_FLAG_STACK8;
// log2 of the highest stack under these flags (0: one tile per walk).
inline int stack_log_of(int flags)
{
    return (flags & FRACTAL_FLAG_STACK8)   ? 3
           : (flags & FRACTAL_FLAG_STACK4) ? 2
           : (flags & FRACTAL_FLAG_STACK2) ? 1
                                           : 0;
}

// Arguments of one register-march launch (FRACTAL_FLAG_MARCH).
struct MarchArgs {
    const uint8_t *src;
    uint8_t *dst;
    int k;
    float alpha;
    int rb;         // block level k - r
    int order;      // FRACTAL_ORDER_*
    uint32_t total; // tiles in the map's id space (3^rb, or 4^rb for BB)
    int band_log;   // log2 of the bands each tile is cut into
    int stack_log;  // lambda map: 0, or c > 0 for stacks of up to 2^c tiles (no bands)
    uint32_t stack_waves; // stacks: wavefronts of the grid (groups x (1 + (3^c - 1) / 2))
};
typedef void (*MarchFn)(MarchArgs);
// Kernel for (map, rule, r, T steps, non-temporal stores); nullptr if none.
// alt: the kernel compiled for the other occupancy where one exists.
MarchFn pick_march(int map, int rule, int r, int T, bool nt, bool alt);
// Lambda-map kernels of 10 or 12 steps (the sizes between 8 and 16 that
// even out a sixteen-step tuning's launches); nullptr if none.
MarchFn pick_march_mid(int rule, int r, int T, bool nt);
// Tiles one wavefront handles (0: no march kernel for this shape).
int march_tiles_per_wave(int rule, int r, int T);
int march_band_log(int rule, int r, int T, uint64_t tiles);
int launch_march(int map, int k, int rule, float alpha, void *b0, void *b1, int steps,
                 const fractal_tuning &t, hipStream_t s);

// The block engines (64 x 64 tiles): one wavefront per tile.
struct BlockArgs {
    const uint8_t *src;
    uint8_t *dst;
    int k;
    float alpha;
    int rb;         // tile level k - 6
    int order;      // FRACTAL_ORDER_* (lambda map)
    uint32_t total; // tiles in the map's id space
    int steps;      // steps this launch advances, 1..16
};
typedef void (*BlockFn)(BlockArgs);
// The automaton's block kernel for launches of up to `depth` steps (16, 24,
// 32 or 36).
BlockFn pick_block_ca(int map, bool nt, int depth);
// The automaton's block kernel on 128 x 128 tiles, two blocks per lane.
BlockFn pick_block2_ca(int map, bool nt);
// The block engine over a batch list (table, entries, tiles, slot, steps).
typedef void (*BatchBlockFn)(const struct BatchEntry *, int, uint64_t, int, int);
// depth: the most steps of one launch of the list's class (16 or 32).
BatchBlockFn pick_batch_block(int rule, bool nt, int depth);
// The block engine over compact storage of 64 x 64 tiles (compact_block.hip).
int launch_compact_block(int k, int rule, float alpha, void *c0, void *c1, int steps, int cap,
                         bool nt, hipStream_t s);
int launch_block(int map, int k, int rule, float alpha, void *b0, void *b1, int steps,
                 const fractal_tuning &t, hipStream_t s);

// Launch `steps` step kernels (validated arguments).
int launch_steps(int map, int k, int rule, float alpha, void *b0, void *b1,
                 int steps, const fractal_tuning &t, hipStream_t s);

// lambda map kernels: per wavefront (ballots or matrix core), and per lane.
int launch_lambda_map(int k, int r, uint32_t *d_xy, bool mfma, hipStream_t s);
int launch_lambda_tiles(int rb, int order, uint32_t *d_xy, hipStream_t s);

// Seeded state fill.
int launch_seed_fill(int k, int rule, uint32_t stream_id, void *d_buf,
                     hipStream_t s);

// Sum of a state's cell bit patterns into *d_out (device uint64), added.
int launch_checksum(int k, int rule, const void *d_buf,
                    unsigned long long *d_out, hipStream_t s);

// Batched steps: device table entry per instance.
struct BatchEntry {
    uint64_t tile_begin; // prefix of 3^(k_j - r) over earlier entries of the list
    uint8_t *buf0;
    uint8_t *buf1;
    int32_t k;
    int32_t r;
    int32_t rule;
    int32_t phase; // buffer holding the state at the start (its parity)
    float alpha;
    int32_t flip0; // launches this instance makes before this list's first
};
static_assert(sizeof(BatchEntry) == 48, "BatchEntry layout");
// An instance sits in at most one list per launch size (16, 8, 4, 2, 1 steps).
constexpr int kMaxListsPerItem = 6; // launch sizes T, T/2, ..., T/32

// One gasket advanced by a batched launch sequence.
struct BatchItem {
    int k, rule;
    int steps; // steps to run in this sequence
    int phase; // input is buf[phase & 1]
    float alpha;
    uint8_t *buf0, *buf1;
    fractal_tuning tuning; // tile launch (r, threads, flags) for this item
    // march classes: take as many T-step launches as fit and the rest in
    // powers of two, whatever the parity of their count (the caller tracks
    // which buffer holds the state: BatchPlan::launches gives the count)
    bool any_parity = false;
};

// Instances grouped by launch class (rule, r, threads, step flags).  A class
// splits each item's steps into launches of T steps (the class's largest),
// then smaller ones: LDS-engine classes give an item 2 floor(steps / 2T)
// T-step launches and single steps for the rest; march classes (which have
// every power of two up to T) take as many T-step launches as fit, the rest
// in powers of two, and split the largest launch in two where the count's
// parity differs from the steps' (so the result lands in buf[steps & 1]),
// except for items marked any_parity.
// A class keeps one list per launch size, largest first, each sorted by how
// many launches of that size an item makes, so the items taking part in any
// launch form a prefix of the list.  Launch slot t runs, per class, launch
// t - (slots of the earlier lists) of the list it falls in.
class BatchPlan {
  public:
    // Fills `host` (capacity >= kMaxListsPerItem * items.size()) and records
    // the classes.
    void build(const std::vector<BatchItem> &items, BatchEntry *host);
    // Launch slot t of every class that has work in it.
    int launch_slot(const BatchEntry *d_table, int t, bool persistent, hipStream_t s) const;
    int slots() const { return slots_; }
    size_t entries() const { return entries_; }
    // Launches item i takes part in (each swaps its two buffers once).
    int launches(size_t i) const { return i < launches_.size() ? launches_[i] : 0; }

  private:
    struct List {
        int T = 1;                    // steps per launch
        size_t first = 0;
        std::vector<int> count;       // per entry: launches it takes part in (descending)
        std::vector<uint64_t> prefix; // tile prefix, size count.size() + 1
        int slots() const { return count.empty() ? 0 : count[0]; }
    };
    struct Class {
        int rule, r, threads, flags;
        std::vector<List> lists;
    };
    std::vector<Class> classes_;
    std::vector<int> launches_;
    int slots_ = 0;
    size_t entries_ = 0;
};

// Launch sizes of `steps` steps on the march engine with at most Tmax steps
// per launch: counts[j] launches of Tmax >> j steps, as many Tmax-step
// launches as fit and the rest in powers of two; with even_parity, a count
// of the parity of `steps` (the largest launch split in two where needed).
void march_split(int steps, int Tmax, int (&counts)[kMaxListsPerItem], bool even_parity = true);

// Deterministic sum of n0 8-byte slots (uint64, or float64 if f64) at the
// start of `work` into *d_out by a fixed 4096-ary tree; `work` must hold
// reduce_tree_words(n0) words.
uint64_t reduce_tree_words(uint64_t n0);
int launch_reduce_tree(uint64_t *work, uint64_t n0, void *d_out, bool f64, hipStream_t s);

// Batched march kernel for (rule, r, T steps, non-temporal stores).
typedef void (*BatchMarchFn)(const BatchEntry *, int, uint64_t, int, int, uint32_t);
BatchMarchFn pick_batch_march_ca(int r, int T, bool nt);
BatchMarchFn pick_batch_march_heat(int r, int T, bool nt);
inline BatchMarchFn pick_batch_march(int rule, int r, int T, bool nt)
{
    return rule == FRACTAL_RULE_CA ? pick_batch_march_ca(r, T, nt)
                                   : pick_batch_march_heat(r, T, nt);
}

// Batched LDS-engine step kernel of one rule for (r, threads, flags): one
// workgroup per tile; nullptr if not instantiated.
typedef void (*TileFn)(const BatchEntry *, int, uint32_t, int);
TileFn pick_batch_ca(int r, int threads, int flags);
TileFn pick_batch_heat(int r, int threads, int flags);

// Tile launch used for one batched instance: `forced` (may be NULL) overrides
// the per-level cached or default tuning.
fractal_tuning batch_item_tuning(int k, int rule, const fractal_tuning *forced);

} // namespace fractal
