// serve.cpp -- request server: continuous batching of gasket simulations
// resident in a caller-provided device arena.
//
// A scheduler thread admits queued requests first come first served when a
// slot and arena space are free, initialises their state on the device (on
// a stream of its own, so that the memory-bound clear and seed of new
// requests overlap the compute-bound steps of the running ones; the step
// stream waits for it only before the iteration that first uses them),
// and then repeatedly enqueues one iteration: steps_per_iter steps of every
// active slot, as the batched plan's fused launches (slots with fewer
// remaining steps drop out of the later launches of the iteration).  Requests that
// arrive meanwhile join the next iteration.  A finished slot leaves the table
// at once; a retire thread waits for its last step, computes nothing on the
// host, copies the final state (if asked) and the checksum back, stamps the
// result and returns the arena range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "serve_sched.hpp"

namespace fractal {

// Steps each admitted request advances per scheduling iteration until
// fractal_serve_set_steps_per_iter changes it: the automaton's longest
// launch (16 steps) then always fits.
constexpr int kDefaultStepsPerIter = 16;

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

namespace {

enum TicketState { QUEUED, ACTIVE, RETIRING, DONE };

struct Ticket {
    fractal_request rq;
    fractal_result res;
    TicketState state;
    size_t bytes; // arena footprint (both buffers)
};

struct Slot {
    bool busy = false;
    uint64_t ticket = 0;
    size_t offset = 0;
    int k = 0, rule = 0, steps = 0, done = 0;
    fractal_tuning tuning = {0, 64, 0, 0};
    float alpha = 0.0f;
    uint8_t *buf0 = nullptr, *buf1 = nullptr;
};

struct RetireJob {
    uint64_t ticket;
    int slot;
    hipEvent_t ready;        // last step and checksum of this slot done
    const uint8_t *final_buf;
    size_t state_bytes;
};

} // namespace

class Server {
  public:
    Server(uint8_t *arena, size_t bytes, int max_slots, int per_iter, hipStream_t s)
        : arena_(arena), arena_bytes_(bytes), max_slots_(max_slots), per_iter_(per_iter),
          stream_(s)
    {
    }

    int init()
    {
        int dev = 0;
        int rc = hip_error(hipGetDevice(&dev), "get device");
        if (rc)
            return rc;
        device_ = dev;
        // header of the arena: two device tables (double-buffered) and the
        // per-slot checksums; the rest holds request states
        const size_t table_bytes = sizeof(BatchEntry) * kMaxListsPerItem * (size_t)(max_slots_ + 1);
        table_off_[0] = 0;
        table_off_[1] = align(table_bytes);
        sums_off_ = table_off_[1] + align(table_bytes);
        const size_t header = align(sums_off_ + sizeof(unsigned long long) * max_slots_);
        if (arena_bytes_ <= header)
            return set_error(FRACTAL_E_NOMEM, "arena of %zu bytes is smaller than the %zu-byte header",
                             arena_bytes_, header);
        state_base_ = header;
        alloc_.reset(arena_bytes_ - header, 256);
        slots_.assign(max_slots_, Slot());
        slot_free_.assign(max_slots_, true);
        for (int i = 0; i < 2; ++i) {
            if ((rc = hip_error(hipHostMalloc((void **)&host_table_[i], table_bytes), "pinned table")))
                return rc;
            if ((rc = hip_error(hipEventCreateWithFlags(&table_ev_[i], hipEventDisableTiming),
                                "event")))
                return rc;
            if ((rc = hip_error(hipEventRecord(table_ev_[i], stream_), "event record")))
                return rc;
        }
        if ((rc = hip_error(hipHostMalloc((void **)&host_sums_, sizeof(unsigned long long) * max_slots_),
                            "pinned sums")))
            return rc;
        if ((rc = hip_error(hipStreamCreateWithFlags(&copy_stream_, hipStreamNonBlocking),
                            "copy stream")))
            return rc;
        if ((rc = hip_error(hipStreamCreateWithFlags(&init_stream_, hipStreamNonBlocking),
                            "init stream")))
            return rc;
        if ((rc = hip_error(hipEventCreateWithFlags(&init_ev_, hipEventDisableTiming), "event")))
            return rc;
        worker_ = std::thread([this] { run(); });
        retirer_ = std::thread([this] { retire_loop(); });
        return FRACTAL_OK;
    }

    ~Server()
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

    int submit(const fractal_request *rq, uint64_t *ticket)
    {
        if (!rq || !ticket)
            return set_error(FRACTAL_E_INVAL, "null request or ticket pointer");
        if (rq->k < 0 || rq->k > kMaxStepLevel)
            return set_error(FRACTAL_E_INVAL, "level k=%d outside [0, %d]", rq->k, kMaxStepLevel);
        if (rq->rule != FRACTAL_RULE_CA && rq->rule != FRACTAL_RULE_HEAT)
            return set_error(FRACTAL_E_INVAL, "unknown rule %d", rq->rule);
        if (rq->steps < 0)
            return set_error(FRACTAL_E_INVAL, "negative step count %d", rq->steps);
        if (rq->rule == FRACTAL_RULE_HEAT &&
            !(rq->alpha > 0.0f && rq->alpha <= 0.25f)) // also rejects NaN
            return set_error(FRACTAL_E_INVAL, "heat coefficient alpha=%g outside (0, 0.25]",
                             (double)rq->alpha);
        const size_t one = align(state_bytes(rq->k, rq->rule));
        const size_t bytes = 2 * one;
        if (!alloc_.fits_ever(bytes))
            return set_error(FRACTAL_E_NOMEM, "request needs %zu bytes, arena holds %zu", bytes,
                             alloc_.capacity());
        std::lock_guard<std::mutex> lk(mu_);
        if (stopping_)
            return set_error(FRACTAL_E_INVAL, "server is shutting down");
        const uint64_t id = ++next_ticket_;
        Ticket t;
        t.rq = *rq;
        std::memset(&t.res, 0, sizeof t.res);
        t.res.t_arrival = rq->t_arrival >= 0.0 ? rq->t_arrival : now_s();
        t.state = QUEUED;
        t.bytes = bytes;
        tickets_[id] = t;
        queue_.push(id, bytes);
        *ticket = id;
        cv_.notify_all();
        return FRACTAL_OK;
    }

    void set_steps_per_iter(int n)
    {
        std::lock_guard<std::mutex> lk(mu_);
        per_iter_ = n;
    }

    int poll(uint64_t ticket, fractal_result *res)
    {
        if (!res)
            return set_error(FRACTAL_E_INVAL, "null result pointer");
        std::lock_guard<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end())
            return set_error(FRACTAL_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
        if (it->second.state != DONE)
            return FRACTAL_E_AGAIN;
        *res = it->second.res;
        tickets_.erase(it);
        return FRACTAL_OK;
    }

    void shutdown()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
            cv_.notify_all();
        }
        if (worker_.joinable())
            worker_.join();
        {
            std::lock_guard<std::mutex> lk(rmu_);
            rstop_ = true;
            rcv_.notify_all();
        }
        if (retirer_.joinable())
            retirer_.join();
    }

  private:
    static size_t align(size_t b) { return (b + 255) / 256 * 256; }

    void fail_ticket(uint64_t id, int code)
    {
        auto it = tickets_.find(id);
        if (it == tickets_.end())
            return;
        it->second.res.status = code;
        it->second.res.t_done = now_s();
        it->second.state = DONE;
    }

    // Scheduler thread.  Slots are read and written under mu_; GPU work is
    // enqueued from snapshots taken under the lock.
    void run()
    {
        (void)hipSetDevice(device_);
        int parity = 0;
        for (;;) {
            std::vector<Admitted> adm;
            std::vector<std::pair<int, Slot>> act; // (slot index, snapshot)
            std::vector<fractal_request> adm_rq;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stopping_ || !queue_.empty() || active_count() > 0; });
                adm = queue_.admit(slot_free_, alloc_);
                if (stopping_ && queue_.empty() && active_count() == 0 && adm.empty())
                    break;
                if (adm.empty() && active_count() == 0) {
                    // queued work waits for a retiring slot to return memory
                    cv_.wait_for(lk, std::chrono::milliseconds(1));
                    continue;
                }
                const double t = now_s();
                for (const Admitted &a : adm) {
                    Ticket &tk = tickets_[a.ticket];
                    tk.state = ACTIVE;
                    tk.res.t_admit = t;
                    Slot &sl = slots_[a.slot];
                    sl.busy = true;
                    sl.ticket = a.ticket;
                    sl.offset = a.offset;
                    sl.k = tk.rq.k;
                    sl.rule = tk.rq.rule;
                    sl.tuning = batch_item_tuning(sl.k, sl.rule, nullptr);
                    sl.steps = tk.rq.steps;
                    sl.done = 0;
                    sl.alpha = tk.rq.alpha;
                    const size_t one = align(state_bytes(sl.k, sl.rule));
                    sl.buf0 = arena_ + state_base_ + a.offset;
                    sl.buf1 = sl.buf0 + one;
                    adm_rq.push_back(tk.rq);
                }
            }
            // initialise admitted states on the device
            for (size_t q = 0; q < adm.size(); ++q) {
                Slot sl = slot_copy(adm[q].slot);
                const fractal_request &rq = adm_rq[q];
                const size_t sb = state_bytes(sl.k, sl.rule);
                int rc = hip_error(hipMemsetAsync(sl.buf1, 0, sb, init_stream_), "state clear");
                if (!rc) {
                    if (rq.h_init)
                        rc = hip_error(hipMemcpyAsync(sl.buf0, rq.h_init, sb, hipMemcpyHostToDevice,
                                                      init_stream_),
                                       "state upload");
                    else
                        rc = launch_seed_fill(sl.k, sl.rule, rq.seed, sl.buf0, init_stream_);
                }
                if (rc)
                    abort_slot(adm[q].slot, rc);
            }
            if (!adm.empty()) {
                // the next launches on the step stream use the new states
                int rc = hip_error(hipEventRecord(init_ev_, init_stream_), "event record");
                if (!rc)
                    rc = hip_error(hipStreamWaitEvent(stream_, init_ev_, 0), "stream wait");
                if (rc)
                    for (const Admitted &a : adm)
                        abort_slot(a.slot, rc);
            }
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (int i = 0; i < max_slots_; ++i)
                    if (slots_[i].busy && slots_[i].done <= slots_[i].steps)
                        act.push_back({i, slots_[i]});
            }
            if (act.empty())
                continue;
            auto rem = [](const Slot &x) { return x.steps - x.done; };
            std::stable_sort(act.begin(), act.end(), [&](const std::pair<int, Slot> &a,
                                                         const std::pair<int, Slot> &b) {
                return rem(a.second) > rem(b.second);
            });
            int per_iter;
            {
                std::lock_guard<std::mutex> lk(mu_);
                per_iter = per_iter_;
            }
            const int c = std::min(per_iter, rem(act[0].second));
            if (c > 0) {
                // the table buffer of two iterations ago must be consumed
                (void)hipEventSynchronize(table_ev_[parity]);
                BatchEntry *ht = host_table_[parity];
                BatchEntry *dt = reinterpret_cast<BatchEntry *>(arena_ + table_off_[parity]);
                std::vector<BatchItem> items;
                items.reserve(act.size());
                for (const auto &a : act) {
                    const Slot &sl = a.second;
                    items.push_back(BatchItem{sl.k, sl.rule, std::min(c, rem(sl)), sl.done, sl.alpha,
                                              sl.buf0, sl.buf1, sl.tuning});
                }
                BatchPlan plan;
                plan.build(items, ht);
                int rc = hip_error(hipMemcpyAsync(dt, ht, sizeof(BatchEntry) * plan.entries(),
                                                  hipMemcpyHostToDevice, stream_),
                                   "table upload");
                for (int j = 0; j < plan.slots() && !rc; ++j)
                    rc = plan.launch_slot(dt, j, false, stream_);
                if (!rc)
                    rc = hip_error(hipEventRecord(table_ev_[parity], stream_), "event record");
                parity ^= 1;
                if (rc) {
                    for (auto &a : act)
                        abort_slot(a.first, rc);
                    continue;
                }
            }
            std::vector<std::pair<int, Slot>> fin;
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (auto &a : act) {
                    Slot &sl = slots_[a.first];
                    sl.done += std::min(c, sl.steps - sl.done);
                    if (sl.done >= sl.steps)
                        fin.push_back({a.first, sl});
                }
            }
            // retire finished slots: checksum on the device, then hand over
            for (auto &f : fin) {
                const int i = f.first;
                const Slot &sl = f.second;
                const uint8_t *final_buf = (sl.steps & 1) ? sl.buf1 : sl.buf0;
                unsigned long long *dsum =
                    reinterpret_cast<unsigned long long *>(arena_ + sums_off_) + i;
                int rc = hip_error(hipMemsetAsync(dsum, 0, sizeof *dsum, stream_), "sum clear");
                if (!rc)
                    rc = launch_checksum(sl.k, sl.rule, final_buf, dsum, stream_);
                hipEvent_t ev = nullptr;
                if (!rc)
                    rc = hip_error(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
                if (!rc)
                    rc = hip_error(hipEventRecord(ev, stream_), "event record");
                if (rc) {
                    if (ev)
                        (void)hipEventDestroy(ev);
                    abort_slot(i, rc);
                    continue;
                }
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    slots_[i].done = slots_[i].steps + 1; // leaves the active set
                    tickets_[sl.ticket].state = RETIRING;
                }
                std::lock_guard<std::mutex> lk(rmu_);
                rq_.push_back(RetireJob{sl.ticket, i, ev, final_buf, state_bytes(sl.k, sl.rule)});
                rcv_.notify_all();
            }
        }
    }

    Slot slot_copy(int i)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return slots_[i];
    }

    int active_count() const
    {
        int c = 0;
        for (const Slot &s : slots_)
            if (s.busy && s.done <= s.steps)
                ++c;
        return c;
    }

    // Give up on a slot after a device error (its ticket reports the error).
    void abort_slot(int i, int code)
    {
        (void)hipStreamSynchronize(init_stream_);
        (void)hipStreamSynchronize(stream_);
        std::lock_guard<std::mutex> lk(mu_);
        Slot &s = slots_[i];
        if (!s.busy)
            return; // already given up
        fail_ticket(s.ticket, code);
        alloc_.release(s.offset);
        s = Slot();
        slot_free_[i] = true;
        cv_.notify_all();
    }

    // Retire thread: wait for a finished slot, copy results, free its range.
    void retire_loop()
    {
        (void)hipSetDevice(device_);
        for (;;) {
            RetireJob job;
            {
                std::unique_lock<std::mutex> lk(rmu_);
                rcv_.wait(lk, [&] { return rstop_ || !rq_.empty(); });
                if (rq_.empty() && rstop_)
                    break;
                job = rq_.front();
                rq_.pop_front();
            }
            int rc = hip_error(hipEventSynchronize(job.ready), "wait for slot");
            (void)hipEventDestroy(job.ready);
            void *h_out = nullptr;
            {
                std::lock_guard<std::mutex> lk(mu_);
                h_out = tickets_[job.ticket].rq.h_out;
            }
            if (!rc && h_out)
                rc = hip_error(hipMemcpyAsync(h_out, job.final_buf, job.state_bytes,
                                              hipMemcpyDeviceToHost, copy_stream_),
                               "state download");
            if (!rc)
                rc = hip_error(hipMemcpyAsync(&host_sums_[job.slot],
                                              reinterpret_cast<unsigned long long *>(arena_ + sums_off_) + job.slot,
                                              sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                              copy_stream_),
                               "checksum download");
            if (!rc)
                rc = hip_error(hipStreamSynchronize(copy_stream_), "copy sync");
            std::lock_guard<std::mutex> lk(mu_);
            Ticket &tk = tickets_[job.ticket];
            tk.res.status = rc;
            tk.res.checksum = rc ? 0 : host_sums_[job.slot];
            tk.res.t_done = now_s();
            tk.state = DONE;
            Slot &s = slots_[job.slot];
            alloc_.release(s.offset);
            s = Slot();
            slot_free_[job.slot] = true;
            cv_.notify_all();
        }
    }

    uint8_t *arena_;
    size_t arena_bytes_;
    int max_slots_, per_iter_;
    hipStream_t stream_, copy_stream_ = nullptr, init_stream_ = nullptr;
    hipEvent_t init_ev_ = nullptr; // the newest admissions' initialisation
    int device_ = 0;
    size_t table_off_[2] = {0, 0}, sums_off_ = 0, state_base_ = 0;
    BatchEntry *host_table_[2] = {nullptr, nullptr};
    hipEvent_t table_ev_[2] = {nullptr, nullptr};
    unsigned long long *host_sums_ = nullptr;

    std::mutex mu_; // tickets_, queue_, alloc_, slot_free_, slot ownership
    std::condition_variable cv_;
    bool stopping_ = false;
    uint64_t next_ticket_ = 0;
    std::unordered_map<uint64_t, Ticket> tickets_;
    AdmissionQueue queue_;
    ArenaAllocator alloc_;
    std::vector<Slot> slots_;
    std::vector<bool> slot_free_;

    std::mutex rmu_;
    std::condition_variable rcv_;
    bool rstop_ = false;
    std::deque<RetireJob> rq_;

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
                           kDefaultStepsPerIter, static_cast<hipStream_t>(stream));
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
    static_cast<Server *>(server)->set_steps_per_iter(steps_per_iter);
    return FRACTAL_OK;
}

int fractal_serve_submit(void *server, const fractal_request *rq, uint64_t *ticket)
{
    if (!server)
        return set_error(FRACTAL_E_INVAL, "null server");
    return static_cast<Server *>(server)->submit(rq, ticket);
}

int fractal_serve_poll(void *server, uint64_t ticket, fractal_result *res)
{
    if (!server)
        return set_error(FRACTAL_E_INVAL, "null server");
    return static_cast<Server *>(server)->poll(ticket, res);
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
