// serve.cpp -- request server: continuous batching of gasket simulations
// resident in a caller-provided device arena.
//
// The scheduling (tickets, FIFO admission by arena space and slot,
// iterations, retirement, statistics) is ServeCore in serve_sched.hpp; this
// file is its device side and its two threads.  The executor initialises
// admitted requests on a stream of its own, so that the memory-bound clear
// and seed of new requests overlap the compute-bound steps of the running
// ones (the step stream waits for it only before the iteration that first
// uses them), enqueues each iteration as the batched plan's fused launches
// over every active slot, and retires a finished slot by a checksum on the
// device, then a copy of the final state and the checksum to the host.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "serve_sched.hpp"

namespace fractal {

// Steps each admitted request advances per scheduling iteration until
// fractal_serve_set_steps_per_iter changes it: the longest batch launch of
// the block engines (32 steps; the march's are 16).
constexpr int kDefaultStepsPerIter = 32;

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

class SteadyClock : public ServeClock {
  public:
    double now() override { return now_s(); }
};

// The arena starts with a header: two device tables (the iteration being
// enqueued and the one before it may still be read) and one checksum per
// slot; request states follow at state_base_.
class HipExecutor : public ServeExecutor {
  public:
    HipExecutor(uint8_t *arena, size_t bytes, int max_slots, hipStream_t s)
        : arena_(arena), arena_bytes_(bytes), max_slots_(max_slots), stream_(s),
          flips_(max_slots > 0 ? max_slots : 0, 0), final_(max_slots > 0 ? max_slots : 0, 0)
    {
        table_bytes_ = sizeof(BatchEntry) * kMaxListsPerItem * (size_t)(max_slots + 1);
        table_off_[0] = 0;
        table_off_[1] = align(table_bytes_);
        sums_off_ = table_off_[1] + align(table_bytes_);
        state_base_ = align(sums_off_ + sizeof(unsigned long long) * (size_t)max_slots);
    }

    ~HipExecutor() override
    {
        for (int i = 0; i < 2; ++i) {
            if (host_table_[i])
                (void)hipHostFree(host_table_[i]);
            if (table_ev_[i])
                (void)hipEventDestroy(table_ev_[i]);
        }
        if (host_sums_)
            (void)hipHostFree(host_sums_);
        if (copy_stream_)
            (void)hipStreamDestroy(copy_stream_);
        if (init_stream_)
            (void)hipStreamDestroy(init_stream_);
        if (init_ev_)
            (void)hipEventDestroy(init_ev_);
    }

    int init()
    {
        if (arena_bytes_ <= state_base_)
            return set_error(FRACTAL_E_NOMEM,
                             "arena of %zu bytes is smaller than the %zu-byte header", arena_bytes_,
                             state_base_);
        int dev = 0;
        int rc = hip_error(hipGetDevice(&dev), "get device");
        if (rc)
            return rc;
        device_ = dev;
        for (int i = 0; i < 2; ++i) {
            if ((rc = hip_error(hipHostMalloc((void **)&host_table_[i], table_bytes_),
                                "pinned table")))
                return rc;
            if ((rc = hip_error(hipEventCreateWithFlags(&table_ev_[i], hipEventDisableTiming),
                                "event")))
                return rc;
            if ((rc = hip_error(hipEventRecord(table_ev_[i], stream_), "event record")))
                return rc;
        }
        if ((rc = hip_error(hipHostMalloc((void **)&host_sums_,
                                          sizeof(unsigned long long) * (size_t)max_slots_),
                            "pinned sums")))
            return rc;
        if ((rc = hip_error(hipStreamCreateWithFlags(&copy_stream_, hipStreamNonBlocking),
                            "copy stream")))
            return rc;
        if ((rc = hip_error(hipStreamCreateWithFlags(&init_stream_, hipStreamNonBlocking),
                            "init stream")))
            return rc;
        return hip_error(hipEventCreateWithFlags(&init_ev_, hipEventDisableTiming), "event");
    }

    int device() const { return device_; }
    size_t state_capacity() const override
    {
        return arena_bytes_ > state_base_ ? arena_bytes_ - state_base_ : 0;
    }

    int init_slot(int slot, const ServeSlot &s, const fractal_request &rq) override
    {
        flips_[slot] = 0;
        const size_t sb = state_bytes(s.k, s.rule);
        uint8_t *b0 = buf(s, 0), *b1 = buf(s, 1);
        int rc = hip_error(hipMemsetAsync(b1, 0, sb, init_stream_), "state clear");
        if (!rc) {
            if (rq.h_init)
                rc = hip_error(hipMemcpyAsync(b0, rq.h_init, sb, hipMemcpyHostToDevice,
                                              init_stream_),
                               "state upload");
            else
                rc = launch_seed_fill(s.k, s.rule, rq.seed, b0, init_stream_);
        }
        return rc;
    }

    int join_init() override
    {
        int rc = hip_error(hipEventRecord(init_ev_, init_stream_), "event record");
        if (!rc)
            rc = hip_error(hipStreamWaitEvent(stream_, init_ev_, 0), "stream wait");
        return rc;
    }

    int run(const std::vector<ServeIterItem> &items) override
    {
        // the table buffer of two iterations ago must have been consumed
        (void)hipEventSynchronize(table_ev_[parity_]);
        BatchEntry *ht = host_table_[parity_];
        BatchEntry *dt = reinterpret_cast<BatchEntry *>(arena_ + table_off_[parity_]);
        std::vector<BatchItem> bi;
        bi.reserve(items.size());
        // an iteration's launches need not come in the parity of its steps
        // (sixteen steps run as one launch, not two of eight): each slot's
        // count of launches so far says which buffer holds its state
        for (const ServeIterItem &it : items) {
            const ServeSlot &s = it.s;
            bi.push_back(BatchItem{s.k, s.rule, it.steps, flips_[it.slot], s.alpha, buf(s, 0),
                                   buf(s, 1), batch_item_tuning(s.k, s.rule, nullptr), true});
        }
        BatchPlan plan;
        plan.build(bi, ht);
        for (size_t i = 0; i < items.size(); ++i)
            flips_[items[i].slot] += plan.launches(i);
        int rc = hip_error(hipMemcpyAsync(dt, ht, sizeof(BatchEntry) * plan.entries(),
                                          hipMemcpyHostToDevice, stream_),
                           "table upload");
        for (int j = 0; j < plan.slots() && !rc; ++j)
            rc = plan.launch_slot(dt, j, false, stream_);
        if (!rc)
            rc = hip_error(hipEventRecord(table_ev_[parity_], stream_), "event record");
        parity_ ^= 1;
        return rc;
    }

    int finish(int slot, const ServeSlot &s, uint64_t *token) override
    {
        final_[slot] = flips_[slot] & 1;
        const uint8_t *final_buf = buf(s, final_[slot]);
        unsigned long long *dsum = sums() + slot;
        int rc = hip_error(hipMemsetAsync(dsum, 0, sizeof *dsum, stream_), "sum clear");
        if (!rc)
            rc = launch_checksum(s.k, s.rule, final_buf, dsum, stream_);
        hipEvent_t ev = nullptr;
        if (!rc)
            rc = hip_error(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
        if (!rc)
            rc = hip_error(hipEventRecord(ev, stream_), "event record");
        if (rc) {
            if (ev)
                (void)hipEventDestroy(ev);
            return rc;
        }
        *token = reinterpret_cast<uint64_t>(ev);
        return FRACTAL_OK;
    }

    int collect(uint64_t token, int slot, const ServeSlot &s, void *h_out,
                uint64_t *checksum) override
    {
        hipEvent_t ev = reinterpret_cast<hipEvent_t>(token);
        int rc = hip_error(hipEventSynchronize(ev), "wait for slot");
        (void)hipEventDestroy(ev);
        if (!rc && h_out)
            rc = hip_error(hipMemcpyAsync(h_out, buf(s, final_[slot]), state_bytes(s.k, s.rule),
                                          hipMemcpyDeviceToHost, copy_stream_),
                           "state download");
        if (!rc)
            rc = hip_error(hipMemcpyAsync(&host_sums_[slot], sums() + slot,
                                          sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                          copy_stream_),
                           "checksum download");
        if (!rc)
            rc = hip_error(hipStreamSynchronize(copy_stream_), "copy sync");
        *checksum = rc ? 0 : host_sums_[slot];
        return rc;
    }

    void drain() override
    {
        (void)hipStreamSynchronize(init_stream_);
        (void)hipStreamSynchronize(stream_);
    }

  private:
    static size_t align(size_t b) { return (b + 255) / 256 * 256; }
    uint8_t *buf(const ServeSlot &s, int which) const
    {
        return arena_ + state_base_ + s.offset + (which ? align(state_bytes(s.k, s.rule)) : 0);
    }
    unsigned long long *sums() const
    {
        return reinterpret_cast<unsigned long long *>(arena_ + sums_off_);
    }

    uint8_t *arena_;
    size_t arena_bytes_;
    int max_slots_;
    hipStream_t stream_, copy_stream_ = nullptr, init_stream_ = nullptr;
    hipEvent_t init_ev_ = nullptr; // the newest admissions' initialisation
    int device_ = 0;
    int parity_ = 0;
    size_t table_bytes_ = 0, table_off_[2] = {0, 0}, sums_off_ = 0, state_base_ = 0;
    BatchEntry *host_table_[2] = {nullptr, nullptr};
    hipEvent_t table_ev_[2] = {nullptr, nullptr};
    unsigned long long *host_sums_ = nullptr;
    // per slot: launches enqueued so far (the state is in buf[flips & 1]),
    // and the buffer of the final state once the slot is finished (set by
    // the scheduler thread in finish, read by the retire thread in collect)
    std::vector<int> flips_, final_;
};

// The executor, the clock, the scheduler core and its two threads.
class Server {
  public:
    Server(uint8_t *arena, size_t bytes, int max_slots, hipStream_t s)
        : ex_(arena, bytes, max_slots, s), max_slots_(max_slots)
    {
    }

    int init()
    {
        int rc = ex_.init();
        if (rc)
            return rc;
        core_.reset(new ServeCore(ex_, clock_, max_slots_, kDefaultStepsPerIter));
        worker_ = std::thread([this] { schedule_loop(); });
        retirer_ = std::thread([this] { retire_loop(); });
        return FRACTAL_OK;
    }

    ServeCore &core() { return *core_; }

    void shutdown()
    {
        if (!core_)
            return;
        core_->stop_scheduling();
        if (worker_.joinable())
            worker_.join();
        core_->stop_retiring();
        if (retirer_.joinable())
            retirer_.join();
    }

  private:
    void schedule_loop()
    {
        (void)hipSetDevice(ex_.device());
        bool waiting = false;
        while (core_->wait_work(waiting, 1))
            waiting = core_->iterate() == ServeCore::WAITING;
    }

    void retire_loop()
    {
        (void)hipSetDevice(ex_.device());
        while (core_->wait_retire())
            (void)core_->retire_one();
    }

    HipExecutor ex_;
    SteadyClock clock_;
    int max_slots_;
    std::unique_ptr<ServeCore> core_;
    std::thread worker_, retirer_;
};

} // namespace fractal

using namespace fractal;

extern "C" {

double fractal_now(void) { return now_s(); }

int fractal_serve_create(void *d_arena, size_t arena_bytes, int max_slots, void *stream,
                         void **server)
{
    if (!d_arena || !server)
        return set_error(FRACTAL_E_INVAL, "null arena or server pointer");
    if (reinterpret_cast<uintptr_t>(d_arena) % 256)
        return set_error(FRACTAL_E_INVAL, "arena must be 256-byte aligned");
    if (max_slots < 1 || max_slots > 4096)
        return set_error(FRACTAL_E_INVAL, "max_slots=%d outside [1, 4096]", max_slots);
    Server *s = new Server(static_cast<uint8_t *>(d_arena), arena_bytes, max_slots,
                           static_cast<hipStream_t>(stream));
    int rc = s->init();
    if (rc) {
        s->shutdown();
        delete s;
        return rc;
    }
    *server = s;
    return FRACTAL_OK;
}

int fractal_serve_set_steps_per_iter(void *server, int steps_per_iter)
{
    if (!server)
        return set_error(FRACTAL_E_INVAL, "null server");
    if (steps_per_iter < 1 || steps_per_iter > 1 << 20)
        return set_error(FRACTAL_E_INVAL, "steps_per_iter=%d outside [1, 2^20]", steps_per_iter);
    static_cast<Server *>(server)->core().set_steps_per_iter(steps_per_iter);
    return FRACTAL_OK;
}

int fractal_serve_submit(void *server, const fractal_request *rq, uint64_t *ticket)
{
    if (!server)
        return set_error(FRACTAL_E_INVAL, "null server");
    if (!rq || !ticket)
        return set_error(FRACTAL_E_INVAL, "null request or ticket pointer");
    const char *msg = "";
    const int rc = static_cast<Server *>(server)->core().submit(*rq, ticket, &msg);
    if (rc)
        return set_error(rc, "request (k=%d rule=%d steps=%d): %s", rq->k, rq->rule, rq->steps,
                         msg);
    return FRACTAL_OK;
}

int fractal_serve_poll(void *server, uint64_t ticket, fractal_result *res)
{
    if (!server)
        return set_error(FRACTAL_E_INVAL, "null server");
    if (!res)
        return set_error(FRACTAL_E_INVAL, "null result pointer");
    const int rc = static_cast<Server *>(server)->core().poll(ticket, res);
    if (rc == FRACTAL_E_INVAL)
        return set_error(rc, "unknown ticket %llu", (unsigned long long)ticket);
    return rc;
}

int fractal_serve_stats(void *server, fractal_serve_report *out)
{
    if (!server || !out)
        return set_error(FRACTAL_E_INVAL, "null server or output");
    static_cast<Server *>(server)->core().stats(out);
    return FRACTAL_OK;
}

int fractal_serve_destroy(void *server)
{
    if (!server)
        return set_error(FRACTAL_E_INVAL, "null server");
    Server *s = static_cast<Server *>(server);
    s->shutdown();
    delete s;
    return FRACTAL_OK;
}

} // extern "C"
