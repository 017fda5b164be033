// batch.hip -- many gaskets of uneven levels advanced by one persistent
// kernel per step.  The tiles of all instances form one work list: instance j
// owns tile ids [tile_begin_j, tile_begin_j + 3^(k_j - r_j)); a tile id is
// turned into (instance, local omega) with the per-instance offset table and
// then into a tile by that instance's lambda.  The T step launches of a
// fractal_batch_step call are captured once into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

#include "device_map.hpp"
#include "device_tile.hpp"
#include "internal.hpp"

namespace fractal {

constexpr int kBatchThreads = 64;
constexpr int kBatchMaxRHeat = 5;
constexpr int kBatchMaxRCa = 6;
constexpr int kBatchLds =
    Geom<RULE_CA, 6>::LDS_BYTES > Geom<RULE_HEAT, 5>::LDS_BYTES ? Geom<RULE_CA, 6>::LDS_BYTES
                                                                 : Geom<RULE_HEAT, 5>::LDS_BYTES;

template <int RULE, int R>
__device__ __forceinline__ void batch_tile(uint8_t *lds, const BatchEntry &e, uint32_t L,
                                           int local_step)
{
    const TileXY t = lambda_wave_curve(L, e.k - R);
    const bool odd = ((e.phase + local_step) & 1) != 0;
    StepParams p;
    p.src = odd ? e.buf1 : e.buf0;
    p.dst = odd ? e.buf0 : e.buf1;
    p.k = e.k;
    p.alpha = e.alpha;
    tile_step<RULE, R, kBatchThreads>(lds, p, t.x << R, t.y << R);
}

// Find the instance owning tile id w: the last of entries [0, count) whose
// range starts at or before w (entries are sorted by tile_begin).
__device__ __forceinline__ int find_instance(const BatchEntry *__restrict__ table, int count,
                                             uint64_t w)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].tile_begin <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void batch_dispatch(uint8_t *lds, const BatchEntry &e, uint32_t L,
                                               int local_step)
{
    if (e.rule == RULE_CA) {
        switch (e.r) {
        case 0: batch_tile<RULE_CA, 0>(lds, e, L, local_step); break;
        case 1: batch_tile<RULE_CA, 1>(lds, e, L, local_step); break;
        case 2: batch_tile<RULE_CA, 2>(lds, e, L, local_step); break;
        case 3: batch_tile<RULE_CA, 3>(lds, e, L, local_step); break;
        case 4: batch_tile<RULE_CA, 4>(lds, e, L, local_step); break;
        case 5: batch_tile<RULE_CA, 5>(lds, e, L, local_step); break;
        default: batch_tile<RULE_CA, 6>(lds, e, L, local_step); break;
        }
    } else {
        switch (e.r) {
        case 0: batch_tile<RULE_HEAT, 0>(lds, e, L, local_step); break;
        case 1: batch_tile<RULE_HEAT, 1>(lds, e, L, local_step); break;
        case 2: batch_tile<RULE_HEAT, 2>(lds, e, L, local_step); break;
        case 3: batch_tile<RULE_HEAT, 3>(lds, e, L, local_step); break;
        case 4: batch_tile<RULE_HEAT, 4>(lds, e, L, local_step); break;
        default: batch_tile<RULE_HEAT, 5>(lds, e, L, local_step); break;
        }
    }
}

// Persistent form: workgroup b handles the contiguous tile ids
// [b*per, (b+1)*per) in order, so tiles that are neighbours in the gasket's
// self-similar order stay on one die and share its L2.  Entries [0, count)
// are the active instances; `total` is the end of the last one's range.
__global__ __launch_bounds__(kBatchThreads) void batch_kernel(
    const BatchEntry *__restrict__ table, int count, uint64_t total, int local_step)
{
    __shared__ __align__(16) uint8_t lds[kBatchLds];
    const uint64_t per = (total + gridDim.x - 1) / gridDim.x;
    const uint64_t w0 = (uint64_t)blockIdx.x * per;
    const uint64_t w1 = w0 + per < total ? w0 + per : total;
    if (w0 >= w1)
        return;
    int j = find_instance(table, count, w0);
    uint64_t next = j + 1 < count ? table[j + 1].tile_begin : ~0ull;
    for (uint64_t w = w0; w < w1; ++w) {
        while (w >= next) {
            ++j;
            next = j + 1 < count ? table[j + 1].tile_begin : ~0ull;
        }
        const BatchEntry e = table[j];
        __syncthreads(); // previous tile's LDS reads are done
        batch_dispatch(lds, e, (uint32_t)(w - e.tile_begin), local_step);
    }
}

// One workgroup per tile of the combined work list (ids laid out per die in
// contiguous ranges, as the lambda step kernels do).
__global__ __launch_bounds__(kBatchThreads) void batch_tile_kernel(
    const BatchEntry *__restrict__ table, int count, uint32_t total, int local_step)
{
    __shared__ __align__(16) uint8_t lds[kBatchLds];
    const uint32_t w = xcd_chunk(blockIdx.x, total);
    const BatchEntry e = table[find_instance(table, count, w)];
    batch_dispatch(lds, e, (uint32_t)(w - e.tile_begin), local_step);
}

int batch_supported_r(int rule, int r)
{
    return r >= 0 && r <= (rule == FRACTAL_RULE_CA ? kBatchMaxRCa : kBatchMaxRHeat);
}

int batch_default_r(int k, int rule)
{
    int r = default_tuning(k, rule).r;
    const int rmax = rule == FRACTAL_RULE_CA ? kBatchMaxRCa : kBatchMaxRHeat;
    if (r > rmax)
        r = rmax;
    if (r > k)
        r = k;
    if (k - r > kMaxBlockLevel)
        r = k - kMaxBlockLevel;
    return r;
}

int batch_grid_size()
{
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = cus * 32; // enough resident single-wave workgroups to cover latency
    }
    return grid;
}

int launch_batch(const BatchEntry *d_table, int count, uint64_t total_tiles, int local_step,
                 int grid, hipStream_t s)
{
    if (count <= 0 || total_tiles == 0)
        return FRACTAL_OK;
    if (grid == 0 && total_tiles < 0x7FFFFFFFull) {
        hipLaunchKernelGGL(batch_tile_kernel, dim3((unsigned)total_tiles), dim3(kBatchThreads), 0,
                           s, d_table, count, (uint32_t)total_tiles, local_step);
        return hip_error(hipGetLastError(), "batch kernel launch");
    }
    if (grid == 0)
        grid = batch_grid_size();
    const uint64_t g = total_tiles < (uint64_t)grid ? total_tiles : (uint64_t)grid;
    hipLaunchKernelGGL(batch_kernel, dim3((unsigned)g), dim3(kBatchThreads), 0, s, d_table,
                       count, total_tiles, local_step);
    return hip_error(hipGetLastError(), "batch kernel launch");
}

// Graphs whose launch may still be running, with what they keep alive.
struct PendingGraph {
    hipGraphExec_t exec;
    hipEvent_t done;
    BatchEntry *host_table; // pinned staging of the table copy
};
static std::mutex g_pending_mu;
static std::vector<PendingGraph> g_pending;

static void reap_pending(bool wait)
{
    std::lock_guard<std::mutex> lk(g_pending_mu);
    std::vector<PendingGraph> keep;
    for (PendingGraph &p : g_pending) {
        if (wait)
            (void)hipEventSynchronize(p.done);
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

extern "C" int fractal_batch_step(const fractal_instance *inst, int count,
                                  const fractal_tuning *tuning, void *stream)
{
    if (count < 0 || count > 65536)
        return set_error(FRACTAL_E_INVAL, "instance count %d outside [0, 65536]", count);
    if (count == 0)
        return FRACTAL_OK;
    if (!inst)
        return set_error(FRACTAL_E_INVAL, "null instance array");
    if (tuning && tuning->r != FRACTAL_R_AUTO && (tuning->r < 0 || tuning->r > kMaxR))
        return set_error(FRACTAL_E_INVAL, "tuning r=%d outside [0, %d]", tuning->r, kMaxR);
    if (tuning && (tuning->flags & ~FRACTAL_FLAG_PERSISTENT))
        return set_error(FRACTAL_E_INVAL, "batch tuning flags 0x%x (only PERSISTENT)",
                         tuning->flags);
    // validate every instance, pick its tile level
    std::vector<int> rs(count);
    int max_steps = 0;
    for (int i = 0; i < count; ++i) {
        const fractal_instance &q = inst[i];
        int r = (tuning && tuning->r != FRACTAL_R_AUTO) ? tuning->r
                                                        : batch_default_r(q.k < 0 ? 0 : q.k, q.rule);
        if (q.k >= 0 && r > q.k)
            r = q.k;
        if (q.rule == FRACTAL_RULE_HEAT && r > kBatchMaxRHeat)
            r = kBatchMaxRHeat;
        if (q.k >= 0 && q.k - r > kMaxBlockLevel)
            r = q.k - kMaxBlockLevel;
        int rc = check_step_args(q.k, r, q.rule, q.alpha, q.d_buf0, q.d_buf1, q.steps);
        if (rc)
            return set_error(rc, "instance %d: %s", i, fractal_last_error());
        rs[i] = r;
        max_steps = std::max(max_steps, q.steps);
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
    if (max_steps == 0)
        return FRACTAL_OK;

    reap_pending(false);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // order by steps (descending) so the instances still running at any step
    // form a prefix of the table
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return inst[a].steps > inst[b].steps; });
    BatchEntry *host = nullptr;
    int rc = hip_error(hipHostMalloc((void **)&host, sizeof(BatchEntry) * (count + 1)),
                       "pinned table");
    if (rc)
        return rc;
    uint64_t acc = 0;
    std::vector<uint64_t> prefix(count + 1);
    for (int i = 0; i < count; ++i) {
        const int src = order[i];
        const fractal_instance &q = inst[src];
        BatchEntry &e = host[i];
        e.tile_begin = acc;
        e.buf0 = static_cast<uint8_t *>(q.d_buf0);
        e.buf1 = static_cast<uint8_t *>(q.d_buf1);
        e.k = q.k;
        e.r = rs[src];
        e.rule = q.rule;
        e.phase = 0;
        e.alpha = q.alpha;
        e.pad = 0;
        prefix[i] = acc;
        acc += pow3_u64(q.k - rs[src]);
    }
    prefix[count] = acc;
    host[count] = BatchEntry{acc, nullptr, nullptr, 0, 0, 0, 0, 0.0f, 0};

    BatchEntry *d_table = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t cs = nullptr;
    // persistent workgroups when asked for, else one workgroup per tile
    const int grid = (tuning && (tuning->flags & FRACTAL_FLAG_PERSISTENT)) ? batch_grid_size() : 0;
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
        if (graph)
            (void)hipGraphDestroy(graph);
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (done)
            (void)hipEventDestroy(done);
        if (d_table)
            (void)hipFreeAsync(d_table, s);
        (void)hipStreamSynchronize(s);
        (void)hipHostFree(host);
        return code;
    };
    if ((rc = hip_error(hipMallocAsync((void **)&d_table, sizeof(BatchEntry) * (count + 1), s),
                        "device table")))
        return fail(rc);
    if ((rc = hip_error(hipMemcpyAsync(d_table, host, sizeof(BatchEntry) * (count + 1),
                                       hipMemcpyHostToDevice, s),
                        "table copy")))
        return fail(rc);
    // capture every step launch into one graph
    if ((rc = hip_error(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream")))
        return fail(rc);
    if ((rc = hip_error(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal),
                        "begin capture")))
        return fail(rc);
    int active = count;
    for (int t = 0; t < max_steps; ++t) {
        while (active > 0 && inst[order[active - 1]].steps <= t)
            --active;
        if ((rc = launch_batch(d_table, active, prefix[active], t, grid, cs)))
            return fail(rc);
    }
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
    if ((rc = hip_error(hipFreeAsync(d_table, s), "table free")))
        return fail(rc);
    d_table = nullptr;
    if ((rc = hip_error(hipEventCreateWithFlags(&done, hipEventDisableTiming), "event")))
        return fail(rc);
    if ((rc = hip_error(hipEventRecord(done, s), "event record")))
        return fail(rc);
    std::lock_guard<std::mutex> lk(g_pending_mu);
    g_pending.push_back(PendingGraph{exec, done, host});
    return FRACTAL_OK;
}
