// batch.hip -- many gaskets of uneven levels advanced together.
//
// Instances are grouped into launch classes by their tile launch (rule, tile
// level r, threads, step flags).  The tiles of a class form one work list:
// instance j owns tile ids [tile_begin_j, tile_begin_j + 3^(k_j - r)); a tile
// id is turned into (instance, local omega) with the per-instance offset
// table and then into a tile by that instance's lambda.  Each launch slot is
// one launch per class (of 1, 2, 4, 8 or 16 steps); the launches of a
// fractal_batch_step call are captured once into a HIP graph.  The device
// table lives in a caller-owned workspace: the library allocates no device
// memory here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace fractal {

// Workgroups of `fn` (256 threads) the whole chip holds at once, a multiple
// of the 8 dies; 0 if the runtime cannot say.
static uint32_t resident_groups(const void *fn)
{
    static std::mutex mu;
    static std::map<const void *, uint32_t> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(fn);
    if (it != cache.end())
        return it->second;
    int dev = 0, cus = 0, per_cu = 0;
    uint32_t g = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) == hipSuccess &&
        cus > 0 && per_cu > 0)
        g = (uint32_t)cus * (uint32_t)per_cu / 8u * 8u;
    cache[fn] = g;
    return g;
}

fractal_tuning batch_item_tuning(int k, int rule, const fractal_tuning *forced)
{
    fractal_tuning t = default_tuning(k, rule);
    if (forced) {
        if (forced->r != FRACTAL_R_AUTO)
            t = tuning_for_r(MAP_LAMBDA, k, rule, forced->r);
        if (forced->threads == 64 || forced->threads == 256)
            t.threads = forced->threads;
        // launch flags apply where any besides the persistent mode are given
        if (forced->flags & ~FRACTAL_FLAG_PERSISTENT)
            t.flags = forced->flags;
    }
    // the batch block kernels take 64 x 64 tiles (heat's 128 x 128 form
    // steps down to them); elsewhere block launches become march launches
    // of the same tile size and step count
    if ((t.flags & FRACTAL_FLAG_BLOCK) && t.r == 7)
        t.r = 6;
    if ((t.flags & FRACTAL_FLAG_BLOCK) && (t.r != 6 || k < 6))
        t.flags = (t.flags & ~FRACTAL_FLAG_BLOCK) | FRACTAL_FLAG_MARCH;
    // a class's launches split into halvings of its largest, so batch block
    // launches take 16 or 32 steps (24 and 36 become 32); the march's
    // longest launch is 16 steps
    if (t.flags & kDeepFlags)
        t.flags = (t.flags & ~kFuseFlags) |
                  ((t.flags & FRACTAL_FLAG_BLOCK) ? FRACTAL_FLAG_FUSE32 : FRACTAL_FLAG_FUSE16);
    if (t.flags & FRACTAL_FLAG_BLOCK)
        t.flags &= ~FRACTAL_FLAG_MARCH;
    t.flags &= FRACTAL_FLAG_SEGMENTS | FRACTAL_FLAG_NT_STORE | FRACTAL_FLAG_MARCH |
               FRACTAL_FLAG_BLOCK | kFuseFlags;
    if (t.flags & (FRACTAL_FLAG_MARCH | FRACTAL_FLAG_BLOCK | kFuseFlags))
        t.flags |= FRACTAL_FLAG_SEGMENTS; // fused, march and block launches move whole segments
    if (t.r > k)
        t.r = k;
    if (t.r > kMaxR)
        t.r = kMaxR;
    if (k - t.r > kMaxBlockLevel)
        t.r = k - kMaxBlockLevel;
    if ((1 << t.r) * (int)cell_bytes(rule) < 16) // fused and march launches need 16-byte rows
        t.flags &= ~(kFuseFlags | FRACTAL_FLAG_MARCH);
    if (!(t.flags & (FRACTAL_FLAG_MARCH | FRACTAL_FLAG_BLOCK)) &&
        (t.flags & (FRACTAL_FLAG_FUSE8 | FRACTAL_FLAG_FUSE16)))
        t.flags = (t.flags & ~kFuseFlags) | FRACTAL_FLAG_FUSE4; // LDS engine: 4 at most
    if ((t.flags & FRACTAL_FLAG_FUSE16) && rule != FRACTAL_RULE_CA && t.r < 4)
        t.flags = (t.flags & ~kFuseFlags) | FRACTAL_FLAG_FUSE8; // narrow heat tiles: 8 at most
    if (t.flags & (FRACTAL_FLAG_MARCH | FRACTAL_FLAG_BLOCK))
        t.threads = 256;
    else if (t.threads == 256 && t.r < 3)
        t.threads = 64;
    t.order = FRACTAL_ORDER_CURVE_XCD;
    return t;
}

void BatchPlan::build(const std::vector<BatchItem> &items, BatchEntry *host)
{
    classes_.clear();
    launches_.assign(items.size(), 0);
    slots_ = 0;
    std::map<std::tuple<int, int, int, int>, std::vector<size_t>> groups;
    for (size_t i = 0; i < items.size(); ++i) {
        const BatchItem &it = items[i];
        groups[std::make_tuple(it.rule, it.tuning.r, it.tuning.threads, it.tuning.flags)]
            .push_back(i);
    }
    size_t at = 0;
    for (auto &g : groups) {
        Class c;
        std::tie(c.rule, c.r, c.threads, c.flags) = g.first;
        const int T = launch_steps_of(c.flags);
        // march and block classes launch every power of two up to T
        const bool march = (c.flags & (FRACTAL_FLAG_MARCH | FRACTAL_FLAG_BLOCK)) != 0;
        // launches per size: counts[j] of T >> j steps (LDS engine: T and 1 only)
        std::vector<std::array<int, kMaxListsPerItem>> counts(items.size());
        for (size_t i : g.second) {
            int cnt[kMaxListsPerItem] = {};
            const int steps = items[i].steps;
            if (march) {
                march_split(steps, T, cnt, !items[i].any_parity);
            } else {
                const int f = T > 1 ? 2 * (steps / (2 * T)) : 0;
                cnt[0] = f;
                cnt[T > 1 ? (T == 2 ? 1 : 2) : 0] += steps - T * f;
            }
            std::copy(cnt, cnt + kMaxListsPerItem, counts[i].begin());
            for (int j = 0; j < kMaxListsPerItem; ++j)
                launches_[i] += cnt[j];
        }
        std::vector<int> before(items.size(), 0); // launches in earlier lists
        for (int j = 0; j < kMaxListsPerItem && (T >> j) >= 1; ++j) {
            List list;
            list.T = T >> j;
            list.first = at;
            std::vector<size_t> ids = g.second;
            std::stable_sort(ids.begin(), ids.end(),
                             [&](size_t a, size_t b) { return counts[a][j] > counts[b][j]; });
            uint64_t acc = 0;
            for (size_t i : ids) {
                if (counts[i][j] <= 0)
                    break;
                const BatchItem &it = items[i];
                BatchEntry &e = host[at++];
                e.tile_begin = acc;
                e.buf0 = it.buf0;
                e.buf1 = it.buf1;
                e.k = it.k;
                e.r = c.r;
                e.rule = it.rule;
                e.phase = it.phase & 1;
                e.alpha = it.alpha;
                e.flip0 = before[i];
                list.count.push_back(counts[i][j]);
                list.prefix.push_back(acc);
                acc += pow3_u64(it.k - c.r);
            }
            list.prefix.push_back(acc);
            for (size_t i : g.second)
                before[i] += counts[i][j];
            if (!list.count.empty())
                c.lists.push_back(std::move(list));
        }
        int total = 0;
        for (const List &l : c.lists)
            total += l.slots();
        slots_ = std::max(slots_, total);
        classes_.push_back(std::move(c));
    }
    entries_ = at;
}

int BatchPlan::launch_slot(const BatchEntry *d_table, int t, bool persistent, hipStream_t s) const
{
    for (const Class &c : classes_) {
        const List *lp = nullptr;
        int j = t; // launch index within the list
        for (const List &l : c.lists) {
            if (j < l.slots()) {
                lp = &l;
                break;
            }
            j -= l.slots();
        }
        if (!lp)
            continue;
        const List &list = *lp;
        size_t active = list.count.size();
        while (active > 0 && list.count[active - 1] <= j)
            --active;
        if (active == 0)
            continue;
        const uint64_t total = list.prefix[active];
        const BatchEntry *tab = d_table + list.first;
        if (c.flags & FRACTAL_FLAG_BLOCK) {
            // one wavefront per tile, four per workgroup
            BatchBlockFn fn = pick_batch_block(c.rule, (c.flags & FRACTAL_FLAG_NT_STORE) != 0,
                                               launch_steps_of(c.flags) > 16 ? 32 : 16);
            if (!fn)
                return set_error(FRACTAL_E_INVAL, "no batch block kernel for flags 0x%x", c.flags);
            const uint64_t groups = (total + 3u) / 4u;
            if (groups > 0xFFFFFFFFull)
                return set_error(FRACTAL_E_INVAL, "batch list of %llu tiles is too long",
                                 (unsigned long long)total);
            hipLaunchKernelGGL(fn, dim3((unsigned)groups), dim3(256), 0, s, tab, (int)active,
                               total, j, list.T);
        } else if (c.flags & FRACTAL_FLAG_MARCH) {
            const bool nt = (c.flags & FRACTAL_FLAG_NT_STORE) != 0;
            BatchMarchFn fn = pick_batch_march(c.rule, c.r, list.T, nt);
            const int P = march_tiles_per_wave(c.rule, c.r, list.T);
            if (!fn || P < 1)
                return set_error(FRACTAL_E_INVAL, "no batch march kernel for rule %d r %d T %d",
                                 c.rule, c.r, list.T);
            const int bl = march_band_log(c.rule, c.r, list.T, total);
            const uint64_t waves = ((total << bl) + (uint64_t)P - 1) / (uint64_t)P;
            const uint64_t groups = (waves + 3) / 4;
            if (groups > 0xFFFFFFFFull)
                return set_error(FRACTAL_E_INVAL, "batch list of %llu tiles is too long",
                                 (unsigned long long)total);
            // persistent: as many workgroups as the chip holds, each walking
            // several items (also where one item per workgroup would exceed
            // the launch limit)
            uint64_t grid = groups;
            const uint32_t res = (persistent || groups > (1u << 24))
                                     ? resident_groups((const void *)fn) : 0u;
            if (res > 0 && res < grid)
                grid = res;
            if (grid > (1u << 24))
                return set_error(FRACTAL_E_INVAL, "batch list of %llu tiles is too long",
                                 (unsigned long long)total);
            hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), 0, s, tab, (int)active, total,
                               bl, j, (uint32_t)groups);
        } else {
            // the LDS engine: one workgroup per tile (persistent applies to
            // march classes only)
            const int flags = list.T > 1 ? c.flags : (c.flags & ~kFuseFlags);
            TileFn tf = c.rule == FRACTAL_RULE_CA ? pick_batch_ca(c.r, c.threads, flags)
                                                  : pick_batch_heat(c.r, c.threads, flags);
            if (!tf)
                return set_error(FRACTAL_E_INVAL, "no batch kernel for r=%d threads=%d flags=%d",
                                 c.r, c.threads, flags);
            if (total >= 0x7FFFFFFFull)
                return set_error(FRACTAL_E_INVAL,
                                 "batch list of %llu tiles is too long for the LDS engine",
                                 (unsigned long long)total);
            const uint32_t gx = total < 65536u ? (uint32_t)total : 65536u;
            const uint32_t gy = (uint32_t)((total + gx - 1) / gx);
            hipLaunchKernelGGL(tf, dim3(gx, gy), dim3(c.threads), 0, s, tab, (int)active,
                               (uint32_t)total, j);
        }
        int rc = hip_error(hipGetLastError(), "batch kernel launch");
        if (rc)
            return rc;
    }
    return FRACTAL_OK;
}

// Graphs whose launch may still be running, with what they keep alive.
struct PendingGraph {
    hipGraphExec_t exec;
    hipEvent_t done;
    BatchEntry *host_table; // pinned staging of the table copy
};
static std::mutex g_pending_mu;
static std::vector<PendingGraph> g_pending;

static void reap_pending()
{
    std::lock_guard<std::mutex> lk(g_pending_mu);
    std::vector<PendingGraph> keep;
    for (PendingGraph &p : g_pending) {
        if (hipEventQuery(p.done) == hipSuccess) {
            (void)hipGraphExecDestroy(p.exec);
            (void)hipEventDestroy(p.done);
            (void)hipHostFree(p.host_table);
        } else {
            keep.push_back(p);
        }
    }
    g_pending.swap(keep);
}

} // namespace fractal

using namespace fractal;

// Device table of a batch of `count` instances: one entry per list of its
// launch class (at most one list per launch size), 256-byte granules.
static size_t batch_table_bytes(int count)
{
    const size_t b = sizeof(BatchEntry) * kMaxListsPerItem * (size_t)count;
    return (b + 255) / 256 * 256;
}

extern "C" int fractal_batch_workspace(int count, size_t *bytes)
{
    if (!bytes)
        return set_error(FRACTAL_E_INVAL, "null output");
    if (count < 0 || count > 65536)
        return set_error(FRACTAL_E_INVAL, "instance count %d outside [0, 65536]", count);
    *bytes = batch_table_bytes(count);
    return FRACTAL_OK;
}

extern "C" int fractal_batch_step(const fractal_instance *inst, int count,
                                  const fractal_tuning *tuning, void *d_work, size_t work_bytes,
                                  void *stream)
{
    if (count < 0 || count > 65536)
        return set_error(FRACTAL_E_INVAL, "instance count %d outside [0, 65536]", count);
    if (count == 0)
        return FRACTAL_OK;
    if (!inst)
        return set_error(FRACTAL_E_INVAL, "null instance array");
    if (!d_work)
        return set_error(FRACTAL_E_INVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_work) % 16)
        return set_error(FRACTAL_E_INVAL, "workspace must be 16-byte aligned");
    if (work_bytes < batch_table_bytes(count))
        return set_error(FRACTAL_E_INVAL, "workspace of %zu bytes, %zu needed", work_bytes,
                         batch_table_bytes(count));
    if (tuning) {
        if (tuning->r != FRACTAL_R_AUTO && (tuning->r < 0 || tuning->r > kMaxR))
            return set_error(FRACTAL_E_INVAL, "tuning r=%d outside [0, %d]", tuning->r, kMaxR);
        if (tuning->threads != 0 && tuning->threads != 64 && tuning->threads != 256)
            return set_error(FRACTAL_E_INVAL, "tuning threads=%d (0, 64 or 256)",
                             tuning->threads);
        const int fuse = tuning->flags & kFuseFlags;
        if ((tuning->flags & ~(FRACTAL_FLAG_PERSISTENT | FRACTAL_FLAG_SEGMENTS |
                               FRACTAL_FLAG_NT_STORE | FRACTAL_FLAG_MARCH | kFuseFlags |
                               kStackFlags | FRACTAL_FLAG_OCC_ALT | FRACTAL_FLAG_BLOCK)) ||
            (fuse & (fuse - 1)))
            return set_error(FRACTAL_E_INVAL, "unknown flags 0x%x", tuning->flags);
    }
    // validate every instance and pick its tile launch
    std::vector<BatchItem> items(count);
    for (int i = 0; i < count; ++i) {
        const fractal_instance &q = inst[i];
        const fractal_tuning t = batch_item_tuning(q.k < 0 ? 0 : q.k, q.rule, tuning);
        int rc = check_step_args(q.k, t.r, q.rule, q.alpha, q.d_buf0, q.d_buf1, q.steps);
        if (rc)
            return set_error(rc, "instance %d: %s", i, fractal_last_error());
        items[i] = BatchItem{q.k,  q.rule, q.steps, 0, q.alpha, static_cast<uint8_t *>(q.d_buf0),
                             static_cast<uint8_t *>(q.d_buf1), t};
    }
    // no two instances may share a buffer
    {
        std::vector<std::pair<uintptr_t, uintptr_t>> spans;
        for (int i = 0; i < count; ++i) {
            const size_t b = state_bytes(inst[i].k, inst[i].rule);
            spans.push_back({(uintptr_t)inst[i].d_buf0, (uintptr_t)inst[i].d_buf0 + b});
            spans.push_back({(uintptr_t)inst[i].d_buf1, (uintptr_t)inst[i].d_buf1 + b});
        }
        std::sort(spans.begin(), spans.end());
        for (size_t i = 1; i < spans.size(); ++i)
            if (spans[i].first < spans[i - 1].second)
                return set_error(FRACTAL_E_INVAL, "instance buffers overlap");
    }
    int max_steps = 0;
    for (const BatchItem &it : items)
        max_steps = std::max(max_steps, it.steps);
    if (max_steps == 0)
        return FRACTAL_OK;
    const bool persistent = tuning && (tuning->flags & FRACTAL_FLAG_PERSISTENT);
    reap_pending();
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchEntry *host = nullptr;
    const size_t cap = kMaxListsPerItem * (size_t)count; // one entry per list of its class
    int rc = hip_error(hipHostMalloc((void **)&host, sizeof(BatchEntry) * cap), "pinned table");
    if (rc)
        return rc;
    BatchPlan plan;
    plan.build(items, host);

    BatchEntry *d_table = static_cast<BatchEntry *>(d_work);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t cs = nullptr;
    auto fail = [&](int code) {
        if (cs) {
            hipGraph_t g2 = nullptr;
            hipStreamCaptureStatus st;
            if (hipStreamIsCapturing(cs, &st) == hipSuccess && st == hipStreamCaptureStatusActive)
                (void)hipStreamEndCapture(cs, &g2);
            if (g2)
                (void)hipGraphDestroy(g2);
            (void)hipStreamDestroy(cs);
        }
        (void)hipStreamSynchronize(s);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (done)
            (void)hipEventDestroy(done);
        (void)hipHostFree(host);
        return code;
    };
    if ((rc = hip_error(hipMemcpyAsync(d_table, host, sizeof(BatchEntry) * plan.entries(),
                                       hipMemcpyHostToDevice, s),
                        "table copy")))
        return fail(rc);
    // capture every step launch into one graph
    if ((rc = hip_error(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream")))
        return fail(rc);
    if ((rc = hip_error(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal),
                        "begin capture")))
        return fail(rc);
    for (int t = 0; t < plan.slots(); ++t)
        if ((rc = plan.launch_slot(d_table, t, persistent, cs)))
            return fail(rc);
    if ((rc = hip_error(hipStreamEndCapture(cs, &graph), "end capture")))
        return fail(rc);
    (void)hipStreamDestroy(cs);
    cs = nullptr;
    if ((rc = hip_error(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate")))
        return fail(rc);
    (void)hipGraphDestroy(graph);
    graph = nullptr;
    if ((rc = hip_error(hipGraphLaunch(exec, s), "graph launch")))
        return fail(rc);
    if ((rc = hip_error(hipEventCreateWithFlags(&done, hipEventDisableTiming), "event")))
        return fail(rc);
    if ((rc = hip_error(hipEventRecord(done, s), "event record")))
        return fail(rc);
    std::lock_guard<std::mutex> lk(g_pending_mu);
    g_pending.push_back(PendingGraph{exec, done, host});
    return FRACTAL_OK;
}
