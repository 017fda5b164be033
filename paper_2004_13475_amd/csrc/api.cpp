// api.cpp -- the C ABI of libfractal: argument validation, error reporting,
// tuning cache, autotuner and the map / step entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace fractal {

static thread_local std::string g_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return FRACTAL_OK;
    return set_error(FRACTAL_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static bool ranges_overlap(const void *a, const void *b, size_t bytes)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

int check_step_args(int k, int r, int rule, float alpha, const void *b0, const void *b1,
                    int steps)
{
    if (k < 0 || k > kMaxStepLevel)
        return set_error(FRACTAL_E_INVAL, "level k=%d outside [0, %d]", k, kMaxStepLevel);
    if (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT)
        return set_error(FRACTAL_E_INVAL, "unknown rule %d", rule);
    if (r != FRACTAL_R_AUTO) {
        if (r < 0 || r > k || r > kMaxR)
            return set_error(FRACTAL_E_INVAL, "tile level r=%d outside [0, min(k=%d, %d)]", r,
                             k, kMaxR);
        if (k - r > kMaxBlockLevel)
            return set_error(FRACTAL_E_INVAL, "block level k-r=%d above %d", k - r,
                             kMaxBlockLevel);
    }
    if (rule == FRACTAL_RULE_HEAT && !(std::isfinite(alpha) && alpha > 0.0f && alpha <= 0.25f))
        return set_error(FRACTAL_E_INVAL, "heat coefficient alpha=%g outside (0, 0.25]",
                         (double)alpha);
    if (steps < 0)
        return set_error(FRACTAL_E_INVAL, "negative step count %d", steps);
    if (!b0 || !b1)
        return set_error(FRACTAL_E_INVAL, "null state buffer");
    if (ranges_overlap(b0, b1, state_bytes(k, rule)))
        return set_error(FRACTAL_E_INVAL, "state buffers overlap");
    const size_t align = rule == FRACTAL_RULE_CA ? 16u : 16u;
    if ((reinterpret_cast<uintptr_t>(b0) | reinterpret_cast<uintptr_t>(b1)) % align)
        return set_error(FRACTAL_E_INVAL, "state buffers must be 16-byte aligned");
    return FRACTAL_OK;
}

static int default_threads(int rule, int r)
{
    // one 16-byte chunk per lane: 256 threads once a tile has >= 256 chunks
    const int row_bytes = (1 << r) * (int)cell_bytes(rule);
    const int chunks = row_bytes >= 16 ? (row_bytes / 16) << r : (1 << r);
    return chunks >= 256 ? 256 : 64;
}

// Launch flags for an explicit tile size: where tile rows span 16 bytes,
// the register-march engine with eight steps per launch (non-temporal stores
// once the state is far beyond the caches, level >= 15); the matrix-core map
// and narrower tiles use the LDS engine with whole segments.
static int default_flags(int map, int k, int rule, int r)
{
    int fl = FRACTAL_FLAG_SEGMENTS;
    if ((1 << r) * (int)cell_bytes(rule) >= 16) {
        if (map == MAP_MFMA)
            fl |= rule == FRACTAL_RULE_CA ? (FRACTAL_FLAG_FUSE2 | FRACTAL_FLAG_NT_STORE)
                                          : FRACTAL_FLAG_FUSE4;
        else
            fl |= FRACTAL_FLAG_MARCH | FRACTAL_FLAG_FUSE8 | (k >= 15 ? FRACTAL_FLAG_NT_STORE : 0);
    }
    return fl;
}

fractal_tuning tuning_for_r(int map, int k, int rule, int r)
{
    fractal_tuning t;
    t.r = r;
    t.flags = default_flags(map, k, rule, r);
    t.threads = (t.flags & FRACTAL_FLAG_MARCH) ? 256 : default_threads(rule, r);
    t.order = map == MAP_BB ? FRACTAL_ORDER_NATURAL : FRACTAL_ORDER_CURVE_XCD;
    return t;
}

static int clamp_r(int k, int r)
{
    if (r > k)
        r = k;
    if (k - r > kMaxBlockLevel)
        r = k - kMaxBlockLevel;
    return r;
}

// Used until the autotuner has run for (device, k, rule): the fastest lambda
// launches measured on MI355X (whole launches, levels 12 to 16), sixteen
// steps per launch:
//   automaton  level >= 14: the block engine (one wavefront per 64 x 64
//              tile, one lane per non-empty 8 x 8 block); below: the register
//              march on 16 x 16 tiles;
//   heat       level >= 13: the block engine; below: the march on 16 x 16
//              tiles (eight steps where the tile is narrower than 16 cells).
// The block engines use plain stores (non-temporal ones measured 1.2-1.6x
// slower for heat, 2-12% slower for the automaton); march launches from
// level 15 non-temporal ones.
static fractal_tuning builtin_default(int k, int rule)
{
    const bool ca = rule == FRACTAL_RULE_CA;
    if (k >= (ca ? 14 : 13)) {
        // the block engine, plain stores, in the curve order (neighbouring
        // tiles share halo blocks in L2; for the automaton below level 16
        // split over the dies), with the deepest halo: a launch costs about
        // the same at 16 or 36 steps (its time goes to moving the tile), so
        // the longest launch is the cheapest per step.  From level 16 both
        // rules take 128 x 128 tiles, two blocks per lane (a tile's halo
        // loaded and stepped once for what would be three 64 x 64 tiles,
        // and fewer instructions per useful block); below, too few of them
        // (2187 at level 14) fill the chip
        fractal_tuning t;
        t.r = k < 16 ? 6 : 7;
        t.threads = 256;
        t.order = (ca && k < 16) ? FRACTAL_ORDER_CURVE_XCD : FRACTAL_ORDER_CURVE;
        t.flags = FRACTAL_FLAG_BLOCK | FRACTAL_FLAG_SEGMENTS | FRACTAL_FLAG_FUSE36;
        return t;
    }
    const int r = clamp_r(k, 4);
    fractal_tuning t = tuning_for_r(MAP_LAMBDA, k, rule, r);
    if (t.flags & FRACTAL_FLAG_MARCH) // heat: 16 steps need tiles of side >= 16
        t.flags = FRACTAL_FLAG_MARCH | FRACTAL_FLAG_SEGMENTS |
                  ((ca || r >= 4) ? FRACTAL_FLAG_FUSE16 : FRACTAL_FLAG_FUSE8);
    return t;
}

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, fractal_tuning> g_tune; // (device, k, rule)
static bool g_tune_env_loaded = false;

static int current_device()
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess)
        d = 0;
    return d;
}

// Name a tuning file gives device `dev`: its product name and architecture
// ("none" where the runtime reports no device, for host-only use).  Tabs
// and newlines are replaced, so the name is one field of a line.
static std::string device_key(int dev)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "none";
    std::string s = std::string(p.name) + "|" + p.gcnArchName;
    for (char &c : s)
        if (c == '\t' || c == '\n' || c == '\r')
            c = ' ';
    return s;
}

static const char *kTuneHeader =
    "# libfractal tuning v1: device\tk\trule\tr\tthreads\torder\tflags";

// Reads `path` into (k, rule) -> tuning for devices named `key`; other
// devices' lines are skipped.  E_INVAL on a malformed line or an invalid
// tuning, E_DEVICE if the file cannot be read.
static int read_tuning_file(const char *path, const std::string &key,
                            std::map<std::pair<int, int>, fractal_tuning> *out)
{
    std::ifstream in(path);
    if (!in)
        return set_error(FRACTAL_E_DEVICE, "cannot read tuning file %s", path);
    std::string line;
    int lineno = 0;
    while (std::getline(in, line)) {
        ++lineno;
        if (line.empty() || line[0] == '#')
            continue;
        std::vector<std::string> f;
        std::stringstream ss(line);
        std::string cell;
        while (std::getline(ss, cell, '\t'))
            f.push_back(cell);
        if (f.size() != 7)
            return set_error(FRACTAL_E_INVAL, "%s:%d: expected 7 tab-separated fields", path,
                             lineno);
        int v[6];
        for (int i = 0; i < 6; ++i) {
            char *end = nullptr;
            const long x = std::strtol(f[i + 1].c_str(), &end, 10);
            if (!end || *end || f[i + 1].empty() || x < -1000000 || x > 1000000)
                return set_error(FRACTAL_E_INVAL, "%s:%d: field %d is not an integer", path,
                                 lineno, i + 2);
            v[i] = (int)x;
        }
        const int k = v[0], rule = v[1];
        if (k < 0 || k > kMaxStepLevel || (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT))
            return set_error(FRACTAL_E_INVAL, "%s:%d: bad level or rule", path, lineno);
        const fractal_tuning t{v[2], v[3], v[4], v[5]};
        if (check_tuning(MAP_LAMBDA, k, rule, &t))
            return set_error(FRACTAL_E_INVAL, "%s:%d: %s", path, lineno, fractal_last_error());
        if (f[0] == key)
            (*out)[std::make_pair(k, rule)] = t;
    }
    return FRACTAL_OK;
}

// Adds a file's entries for the current device to the cache.
static int load_tuning_locked(const char *path)
{
    const int dev = current_device();
    std::map<std::pair<int, int>, fractal_tuning> got;
    const int rc = read_tuning_file(path, device_key(dev), &got);
    if (rc)
        return rc;
    for (const auto &e : got)
        g_tune[std::make_tuple(dev, e.first.first, e.first.second)] = e.second;
    return FRACTAL_OK;
}

// Writes the whole cache (every device) to `path` through a temporary file.
static int save_tuning_locked(const char *path)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out)
            return set_error(FRACTAL_E_DEVICE, "cannot write tuning file %s", tmp.c_str());
        out << kTuneHeader << "\n";
        for (const auto &e : g_tune) {
            const fractal_tuning &t = e.second;
            out << device_key(std::get<0>(e.first)) << "\t" << std::get<1>(e.first) << "\t"
                << std::get<2>(e.first) << "\t" << t.r << "\t" << t.threads << "\t" << t.order
                << "\t" << t.flags << "\n";
        }
        if (!out)
            return set_error(FRACTAL_E_DEVICE, "write error on %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return set_error(FRACTAL_E_DEVICE, "cannot rename %s to %s", tmp.c_str(), path);
    return FRACTAL_OK;
}

// FRACTAL_TUNING_FILE, if set, names a tuning file read before the first
// lookup (once per process; a missing or malformed file is ignored) and
// rewritten after every autotuner run.
static const char *env_tuning_file()
{
    const char *p = std::getenv("FRACTAL_TUNING_FILE");
    return (p && *p) ? p : nullptr;
}

static void load_env_tuning_locked()
{
    if (g_tune_env_loaded)
        return;
    g_tune_env_loaded = true;
    if (const char *p = env_tuning_file()) {
        const std::string saved = g_error;
        (void)load_tuning_locked(p);
        g_error = saved;
    }
}

fractal_tuning default_tuning(int k, int rule)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tuning_locked();
    auto it = g_tune.find(std::make_tuple(current_device(), k, rule));
    if (it != g_tune.end())
        return it->second;
    return builtin_default(k, rule);
}

int check_tuning(int map, int k, int rule, const fractal_tuning *t)
{
    if (!t)
        return set_error(FRACTAL_E_INVAL, "null tuning");
    if (map != MAP_LAMBDA && map != MAP_BB && map != MAP_MFMA)
        return set_error(FRACTAL_E_INVAL, "unknown map %d", map);
    if (t->r < 0 || t->r > k || t->r > kMaxR || k - t->r > kMaxBlockLevel)
        return set_error(FRACTAL_E_INVAL, "tuning r=%d invalid for k=%d", t->r, k);
    if (t->threads != 64 && t->threads != 256)
        return set_error(FRACTAL_E_INVAL, "threads=%d must be 64 or 256", t->threads);
    if (t->order < FRACTAL_ORDER_NATURAL || t->order > FRACTAL_ORDER_CURVE_XCD)
        return set_error(FRACTAL_E_INVAL, "unknown order %d", t->order);
    const int fuse = t->flags & kFuseFlags;
    const bool march = (t->flags & FRACTAL_FLAG_MARCH) != 0;
    const int stack = t->flags & kStackFlags;
    if (t->flags & ~(FRACTAL_FLAG_SEGMENTS | FRACTAL_FLAG_NT_STORE | FRACTAL_FLAG_MARCH |
                     kFuseFlags | kStackFlags | FRACTAL_FLAG_OCC_ALT | FRACTAL_FLAG_BLOCK))
        return set_error(FRACTAL_E_INVAL, "unknown flags 0x%x", t->flags);
    if (t->flags & FRACTAL_FLAG_BLOCK) {
        if (t->flags & (FRACTAL_FLAG_MARCH | kStackFlags | FRACTAL_FLAG_OCC_ALT))
            return set_error(FRACTAL_E_INVAL,
                             "FRACTAL_FLAG_BLOCK excludes MARCH, STACK and OCC_ALT");
        if ((t->r != 6 && t->r != 7) || map == MAP_MFMA)
            return set_error(FRACTAL_E_INVAL,
                             "the block engine runs on 64 x 64 or 128 x 128 tiles (r = 6 or 7), "
                             "lambda or BB map");
        if (!(t->flags & FRACTAL_FLAG_SEGMENTS))
            return set_error(FRACTAL_E_INVAL, "block launches need FRACTAL_FLAG_SEGMENTS");
        if (fuse & (fuse - 1))
            return set_error(FRACTAL_E_INVAL, "the FUSE flags are exclusive");
        if (t->threads != 256)
            return set_error(FRACTAL_E_INVAL, "block launches take 256 threads");
        return FRACTAL_OK;
    }
    if (fuse & kDeepFlags)
        return set_error(FRACTAL_E_INVAL, "FUSE24, FUSE32 and FUSE36 need FRACTAL_FLAG_BLOCK");
    if (fuse & (fuse - 1))
        return set_error(FRACTAL_E_INVAL, "the FUSE flags are exclusive");
    if (stack & (stack - 1))
        return set_error(FRACTAL_E_INVAL, "the STACK flags are exclusive");
    if (stack && !march)
        return set_error(FRACTAL_E_INVAL, "STACK flags need FRACTAL_FLAG_MARCH");
    if ((t->flags & FRACTAL_FLAG_OCC_ALT) && !march)
        return set_error(FRACTAL_E_INVAL, "FRACTAL_FLAG_OCC_ALT needs FRACTAL_FLAG_MARCH");
    if ((fuse & (FRACTAL_FLAG_FUSE8 | FRACTAL_FLAG_FUSE16)) && !march)
        return set_error(FRACTAL_E_INVAL, "FUSE8 and FUSE16 need FRACTAL_FLAG_MARCH");
    if ((fuse & FRACTAL_FLAG_FUSE16) && rule != FRACTAL_RULE_CA && t->r < 4)
        return set_error(FRACTAL_E_INVAL, "heat FUSE16 needs tiles of side >= 16");
    if ((fuse || march) && !(t->flags & FRACTAL_FLAG_SEGMENTS))
        return set_error(FRACTAL_E_INVAL, "fused and march launches need FRACTAL_FLAG_SEGMENTS");
    if ((fuse || march) && ((1 << t->r) * (int)cell_bytes(rule)) < 16)
        return set_error(FRACTAL_E_INVAL,
                         "fused and march launches need tile rows of >= 16 bytes");
    if (march && map == MAP_MFMA)
        return set_error(FRACTAL_E_INVAL, "the matrix-core map has no march form");
    if (t->threads == 256 && t->r < 3 && !march)
        return set_error(FRACTAL_E_INVAL, "256 threads need tiles of side >= 8");
    return FRACTAL_OK;
}

static int step_entry(int map, int k, int r, int rule, float alpha, void *b0, void *b1,
                      int steps, void *stream)
{
    int rc = check_step_args(k, r, rule, alpha, b0, b1, steps);
    if (rc)
        return rc;
    fractal_tuning t;
    if (r == FRACTAL_R_AUTO) {
        t = default_tuning(k, rule);
        // the tuned lambda launch fixes the tile size; the bounding box and
        // the matrix-core map take their own launch form at that size (the
        // matrix-core map has no march form)
        if (map != MAP_LAMBDA)
            t = tuning_for_r(map, k, rule, t.r);
    } else {
        t = tuning_for_r(map, k, rule, r);
    }
    if (map == MAP_MFMA && k - t.r > 16)
        return set_error(FRACTAL_E_INVAL, "matrix-core lambda needs k-r <= 16");
    if (steps == 0)
        return FRACTAL_OK;
    return launch_steps(map, k, rule, alpha, b0, b1, steps, t, static_cast<hipStream_t>(stream));
}

} // namespace fractal

using namespace fractal;

extern "C" {

const char *fractal_last_error(void) { return g_error.c_str(); }

int fractal_grid_dims(int k, int r, uint32_t *gx, uint32_t *gy)
{
    if (!gx || !gy)
        return set_error(FRACTAL_E_INVAL, "null output pointer");
    if (k < 0 || k > 40 || r < 0 || r > k)
        return set_error(FRACTAL_E_INVAL, "need 0 <= r <= k <= 40 (k=%d r=%d)", k, r);
    const int rb = k - r;
    *gx = (uint32_t)pow3_u64((rb + 1) / 2);
    *gy = (uint32_t)pow3_u64(rb / 2);
    return FRACTAL_OK;
}

static int map_entry(int k, int r, uint32_t *d_xy, void *stream, bool mfma)
{
    if (!d_xy)
        return set_error(FRACTAL_E_INVAL, "null output buffer");
    if (k < 0 || r < 0 || r > k || k - r > 30)
        return set_error(FRACTAL_E_INVAL, "need 0 <= r <= k and k-r <= 30 (k=%d r=%d)", k, r);
    if (mfma && k - r > 16)
        return set_error(FRACTAL_E_INVAL, "matrix-core lambda needs k-r <= 16 (got %d)", k - r);
    return launch_lambda_map(k, r, d_xy, mfma, static_cast<hipStream_t>(stream));
}

int fractal_lambda_map(int k, int r, uint32_t *d_xy, void *stream)
{
    return map_entry(k, r, d_xy, stream, false);
}

int fractal_lambda_map_mfma(int k, int r, uint32_t *d_xy, void *stream)
{
    return map_entry(k, r, d_xy, stream, true);
}

int fractal_lambda_map_tiles(int k, int r, int order, uint32_t *d_xy, void *stream)
{
    if (!d_xy)
        return set_error(FRACTAL_E_INVAL, "null output buffer");
    if (k < 0 || r < 0 || r > k || k - r > 20)
        return set_error(FRACTAL_E_INVAL, "need 0 <= r <= k and k-r <= 20 (k=%d r=%d)", k, r);
    if (order < FRACTAL_ORDER_NATURAL || order > FRACTAL_ORDER_CURVE_XCD)
        return set_error(FRACTAL_E_INVAL, "unknown order %d", order);
    return launch_lambda_tiles(k - r, order, d_xy, static_cast<hipStream_t>(stream));
}

int fractal_seed_fill(int k, int rule, uint32_t stream_id, void *d_buf, void *stream)
{
    if (k < 0 || k > kMaxStepLevel)
        return set_error(FRACTAL_E_INVAL, "level k=%d outside [0, %d]", k, kMaxStepLevel);
    if (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT)
        return set_error(FRACTAL_E_INVAL, "unknown rule %d", rule);
    if (!d_buf)
        return set_error(FRACTAL_E_INVAL, "null buffer");
    if (reinterpret_cast<uintptr_t>(d_buf) % 16)
        return set_error(FRACTAL_E_INVAL, "buffer must be 16-byte aligned");
    return launch_seed_fill(k, rule, stream_id, d_buf, static_cast<hipStream_t>(stream));
}

int fractal_bb_step(int k, int r, int rule, float alpha, void *d_buf0, void *d_buf1, int steps,
                    void *stream)
{
    return step_entry(MAP_BB, k, r, rule, alpha, d_buf0, d_buf1, steps, stream);
}

int fractal_lambda_step(int k, int r, int rule, float alpha, void *d_buf0, void *d_buf1,
                        int steps, void *stream)
{
    return step_entry(MAP_LAMBDA, k, r, rule, alpha, d_buf0, d_buf1, steps, stream);
}

int fractal_lambda_step_mfma(int k, int r, int rule, float alpha, void *d_buf0, void *d_buf1,
                             int steps, void *stream)
{
    return step_entry(MAP_MFMA, k, r, rule, alpha, d_buf0, d_buf1, steps, stream);
}

int fractal_step_tuned(int map, int k, int rule, float alpha, void *d_buf0, void *d_buf1,
                       int steps, const fractal_tuning *tuning, void *stream)
{
    int rc = check_tuning(map, k, rule, tuning);
    if (rc)
        return rc;
    rc = check_step_args(k, tuning->r, rule, alpha, d_buf0, d_buf1, steps);
    if (rc)
        return rc;
    if (map == MAP_MFMA && k - tuning->r > 16)
        return set_error(FRACTAL_E_INVAL, "matrix-core lambda needs k-r <= 16");
    if (steps == 0)
        return FRACTAL_OK;
    return launch_steps(map, k, rule, alpha, d_buf0, d_buf1, steps, *tuning,
                        static_cast<hipStream_t>(stream));
}

int fractal_get_tuning(int k, int rule, fractal_tuning *out)
{
    if (!out)
        return set_error(FRACTAL_E_INVAL, "null output");
    if (k < 0 || k > kMaxStepLevel || (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT))
        return set_error(FRACTAL_E_INVAL, "bad level or rule");
    *out = default_tuning(k, rule);
    return FRACTAL_OK;
}

int fractal_set_tuning(int k, int rule, const fractal_tuning *t)
{
    if (k < 0 || k > kMaxStepLevel || (rule != FRACTAL_RULE_CA && rule != FRACTAL_RULE_HEAT))
        return set_error(FRACTAL_E_INVAL, "bad level or rule");
    int rc = check_tuning(MAP_LAMBDA, k, rule, t);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tuning_locked();
    g_tune[std::make_tuple(current_device(), k, rule)] = *t;
    return FRACTAL_OK;
}

int fractal_tuning_save(const char *path)
{
    if (!path || !*path)
        return set_error(FRACTAL_E_INVAL, "null or empty path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tuning_locked();
    return save_tuning_locked(path);
}

int fractal_tuning_load(const char *path)
{
    if (!path || !*path)
        return set_error(FRACTAL_E_INVAL, "null or empty path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tuning_locked();
    return load_tuning_locked(path);
}

int fractal_autotune(int k, int rule, float alpha, void *d_buf0, void *d_buf1, void *stream,
                     fractal_tuning *out)
{
    int rc = check_step_args(k, FRACTAL_R_AUTO, rule, alpha, d_buf0, d_buf1, 0);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if ((rc = hip_error(hipEventCreate(&e0), "event create")))
        return rc;
    if ((rc = hip_error(hipEventCreate(&e1), "event create"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    // Few-step timings; enough launches that per-launch gaps are included.
    const int reps = k >= 15 ? 32 : 64; // multiples of 32 (pairs of 16-step launches)
    fractal_tuning best{};
    float best_ms = 1e30f;
    std::vector<fractal_tuning> cands;
    for (int r = 0; r <= kMaxR && r <= k; ++r) {
        if (k - r > kMaxBlockLevel)
            continue;
        const int row_bytes = (1 << r) * (int)cell_bytes(rule);
        if (row_bytes < 16 && k >= 8)
            continue; // tiles below one 16-byte chunk per row are never faster here
        for (int th : {64, 256}) {
            if (th == 256 && r < 4)
                continue;
            for (int order : {FRACTAL_ORDER_NATURAL, FRACTAL_ORDER_CURVE_XCD})
                for (int fl : {0, 1, 3, 9, 11, 17, 19}) {
                    fractal_tuning t{r, th, order, fl};
                    if (fl > 3 && row_bytes < 16)
                        continue;
                    cands.push_back(t);
                }
        }
        // register march: 1, 2, 4, 8 or 16 steps per launch, with and
        // without non-temporal stores; the longer launches also on stacks
        if (row_bytes >= 16)
            for (int fuse : {0, (int)FRACTAL_FLAG_FUSE2, (int)FRACTAL_FLAG_FUSE4,
                             (int)FRACTAL_FLAG_FUSE8, (int)FRACTAL_FLAG_FUSE16})
                for (int nt : {0, (int)FRACTAL_FLAG_NT_STORE})
                    for (int stack : {0, (int)FRACTAL_FLAG_STACK2, (int)FRACTAL_FLAG_STACK4})
                        if ((fuse != FRACTAL_FLAG_FUSE16 || rule == FRACTAL_RULE_CA || r >= 4) &&
                            (stack == 0 || fuse == FRACTAL_FLAG_FUSE8 ||
                             fuse == FRACTAL_FLAG_FUSE16))
                            for (int occ : {0, (int)FRACTAL_FLAG_OCC_ALT})
                                if (occ == 0 || ((fuse == FRACTAL_FLAG_FUSE8 ||
                                                  (fuse == FRACTAL_FLAG_FUSE16 &&
                                                   rule == FRACTAL_RULE_CA)) &&
                                                 r >= 4 && r <= 6))
                                    cands.push_back(fractal_tuning{
                                        r, 256, FRACTAL_ORDER_CURVE_XCD,
                                        FRACTAL_FLAG_MARCH | FRACTAL_FLAG_SEGMENTS | nt | fuse |
                                            stack | occ});
        // 64 x 64 and 128 x 128 tiles (two blocks per lane): the block
        // engine, 8 to 36 steps per launch, every order, with and without
        // non-temporal stores
        if (r == 6 || r == 7)
            for (int fuse : {(int)FRACTAL_FLAG_FUSE8, (int)FRACTAL_FLAG_FUSE16,
                             (int)FRACTAL_FLAG_FUSE24, (int)FRACTAL_FLAG_FUSE32,
                             (int)FRACTAL_FLAG_FUSE36})
                for (int nt : {0, (int)FRACTAL_FLAG_NT_STORE})
                    for (int order : {FRACTAL_ORDER_NATURAL, FRACTAL_ORDER_CURVE,
                                      FRACTAL_ORDER_CURVE_XCD})
                        cands.push_back(fractal_tuning{
                            r, 256, order, FRACTAL_FLAG_BLOCK | FRACTAL_FLAG_SEGMENTS | fuse | nt});
    }
    for (const fractal_tuning &t : cands) {
        // warm-up (even count keeps the state in buf0)
        rc = launch_steps(MAP_LAMBDA, k, rule, alpha, d_buf0, d_buf1, 32, t, s);
        if (!rc)
            rc = hip_error(hipEventRecord(e0, s), "event record");
        if (!rc)
            rc = launch_steps(MAP_LAMBDA, k, rule, alpha, d_buf0, d_buf1, reps, t, s);
        if (!rc)
            rc = hip_error(hipEventRecord(e1, s), "event record");
        if (!rc)
            rc = hip_error(hipEventSynchronize(e1), "event sync");
        float ms = 0.0f;
        if (!rc)
            rc = hip_error(hipEventElapsedTime(&ms, e0, e1), "event time");
        if (rc)
            break;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc)
        return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_env_tuning_locked();
        g_tune[std::make_tuple(current_device(), k, rule)] = best;
        if (const char *p = env_tuning_file())
            if ((rc = save_tuning_locked(p)))
                return rc;
    }
    if (out)
        *out = best;
    return FRACTAL_OK;
}

} // extern "C"
