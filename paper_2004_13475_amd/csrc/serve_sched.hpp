// serve_sched.hpp -- host-only scheduling of the request server: a
// first-fit arena allocator with coalescing, a FIFO admission queue, and the
// scheduler core (tickets, admission, slots, iterations, retirement, latency
// statistics) that drives the device through an executor interface and
// reads time from a clock interface.  No HIP here, so the whole scheduling
// logic is unit-tested on the CPU with a plain compiler, a fake executor and
// a fake clock.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/fractal.h"

namespace fractal {

// Sub-allocates [0, capacity) in multiples of `align` bytes.  First fit over
// the free ranges in address order; freed ranges merge with free neighbours.
class ArenaAllocator {
  public:
    ArenaAllocator(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

    void reset(size_t capacity, size_t align)
    {
        align_ = align ? align : 1;
        capacity_ = capacity / align_ * align_;
        free_.clear();
        used_.clear();
        if (capacity_)
            free_[0] = capacity_;
        in_use_ = 0;
    }

    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }
    size_t capacity() const { return capacity_; }
    size_t in_use() const { return in_use_; }
    bool fits_ever(size_t bytes) const { return round(bytes) <= capacity_; }

    // Returns true and the offset on success; false if no free range fits.
    bool alloc(size_t bytes, size_t *offset)
    {
        const size_t need = round(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > need)
                    free_[off + need] = len - need;
                used_[off] = need;
                in_use_ += need;
                *offset = off;
                return true;
            }
        }
        return false;
    }

    // Returns false for an offset that is not allocated.
    bool release(size_t offset)
    {
        auto u = used_.find(offset);
        if (u == used_.end())
            return false;
        size_t off = offset, len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }

    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &f : free_)
            m = f.second > m ? f.second : m;
        return m;
    }

  private:
    size_t align_ = 256, capacity_ = 0, in_use_ = 0;
    std::map<size_t, size_t> free_; // offset -> length
    std::map<size_t, size_t> used_; // offset -> length
};

// First-come-first-served admission: the head of the queue is admitted as
// soon as a slot and arena space for it are free; nothing behind it is
// admitted first (no skip-ahead), so a large request cannot starve.
struct PendingRequest {
    uint64_t ticket;
    size_t bytes; // arena footprint
};

struct Admitted {
    uint64_t ticket;
    size_t offset;
    int slot;
};

class AdmissionQueue {
  public:
    void push(uint64_t ticket, size_t bytes) { q_.push_back(PendingRequest{ticket, bytes}); }
    bool empty() const { return q_.empty(); }
    size_t size() const { return q_.size(); }

    // Admit from the head while possible.  `slot_free[i]` marks free slots;
    // admitted requests take the lowest free slot.
    std::vector<Admitted> admit(std::vector<bool> &slot_free, ArenaAllocator &arena)
    {
        std::vector<Admitted> out;
        while (!q_.empty()) {
            int slot = -1;
            for (size_t i = 0; i < slot_free.size(); ++i)
                if (slot_free[i]) {
                    slot = (int)i;
                    break;
                }
            if (slot < 0)
                break;
            size_t off = 0;
            if (!arena.alloc(q_.front().bytes, &off))
                break;
            slot_free[slot] = false;
            out.push_back(Admitted{q_.front().ticket, off, slot});
            q_.pop_front();
        }
        return out;
    }

  private:
    std::deque<PendingRequest> q_;
};

// ------------------------------------------------------------ scheduler core

// One admitted request as the scheduler tracks it.
struct ServeSlot {
    bool busy = false;
    uint64_t ticket = 0;
    size_t offset = 0; // arena offset of the request's two state buffers
    int k = 0, rule = 0, steps = 0;
    int done = 0; // steps enqueued so far; steps + 1 once handed to retirement
    float alpha = 0.0f;
};

// One slot's share of a scheduling iteration: `steps` steps from step `done`.
struct ServeIterItem {
    int slot;
    ServeSlot s;
    int steps;
};

// The device side of the server.  Calls come from the scheduler thread
// (init_slot, join_init, run, finish, drain) and the retire thread
// (collect); none is made with the scheduler's lock held.  Every call
// returns a FRACTAL_* status.
class ServeExecutor {
  public:
    virtual ~ServeExecutor() = default;
    // Bytes of the arena left for request states after the executor's own
    // header (device tables, checksums).
    virtual size_t state_capacity() const = 0;
    // Enqueue the initial state of an admitted request in its arena range:
    // rq.h_init uploaded, or the seeded state; the second buffer cleared.
    virtual int init_slot(int slot, const ServeSlot &s, const fractal_request &rq) = 0;
    // Order every later iteration after the initialisations enqueued so far.
    virtual int join_init() = 0;
    // Enqueue one iteration over the given slots.
    virtual int run(const std::vector<ServeIterItem> &items) = 0;
    // Enqueue what a finished slot needs before it retires (its checksum)
    // and return a token for collect().
    virtual int finish(int slot, const ServeSlot &s, uint64_t *token) = 0;
    // Wait for the token's work, copy the final state to h_out (if not
    // NULL) and return its checksum.  The token is released either way.
    virtual int collect(uint64_t token, int slot, const ServeSlot &s, void *h_out,
                        uint64_t *checksum) = 0;
    // Wait for all enqueued work (after a failure, before ranges are reused).
    virtual void drain() = 0;
};

class ServeClock {
  public:
    virtual ~ServeClock() = default;
    virtual double now() = 0; // seconds, monotonic
};

// Request footprint in the arena: two state buffers of 4^k cells, each
// rounded to 256 bytes.
inline size_t serve_footprint(int k, int rule)
{
    const size_t one = ((size_t)1 << (2 * k)) * (rule == FRACTAL_RULE_CA ? 1u : 4u);
    return 2 * ((one + 255) / 256 * 256);
}

// Tickets, FIFO admission by arena space and slot, continuous batching in
// iterations of at most steps_per_iter steps per request, retirement and
// latency statistics.  Thread-safe; iterate() and retire_one() do one unit
// of work each and are what the server's two threads call in a loop (tests
// call them directly).
class ServeCore {
  public:
    static constexpr int kMaxLevel = 16;

    ServeCore(ServeExecutor &ex, ServeClock &clock, int max_slots, int steps_per_iter)
        : ex_(ex), clock_(clock), per_iter_(steps_per_iter)
    {
        alloc_.reset(ex.state_capacity(), 256);
        slots_.assign(max_slots, ServeSlot());
        slot_free_.assign(max_slots, true);
    }

    void set_steps_per_iter(int n)
    {
        std::lock_guard<std::mutex> lk(mu_);
        per_iter_ = n;
    }

    // Validate and queue a request.  *msg names the problem on failure.
    int submit(const fractal_request &rq, uint64_t *ticket, const char **msg)
    {
        *msg = "";
        if (rq.k < 0 || rq.k > kMaxLevel)
            return (*msg = "level outside [0, 16]", FRACTAL_E_INVAL);
        if (rq.rule != FRACTAL_RULE_CA && rq.rule != FRACTAL_RULE_HEAT)
            return (*msg = "unknown rule", FRACTAL_E_INVAL);
        if (rq.steps < 0)
            return (*msg = "negative step count", FRACTAL_E_INVAL);
        if (rq.rule == FRACTAL_RULE_HEAT && !(rq.alpha > 0.0f && rq.alpha <= 0.25f))
            return (*msg = "heat coefficient alpha outside (0, 0.25]", FRACTAL_E_INVAL);
        const size_t bytes = serve_footprint(rq.k, rq.rule);
        std::lock_guard<std::mutex> lk(mu_);
        if (!alloc_.fits_ever(bytes))
            return (*msg = "request larger than the arena", FRACTAL_E_NOMEM);
        if (stopping_)
            return (*msg = "server is shutting down", FRACTAL_E_INVAL);
        const uint64_t id = ++next_ticket_;
        Ticket t;
        t.rq = rq;
        std::memset(&t.res, 0, sizeof t.res);
        t.res.t_arrival = rq.t_arrival >= 0.0 ? rq.t_arrival : clock_.now();
        t.state = QUEUED;
        tickets_[id] = t;
        queue_.push(id, bytes);
        ++submitted_;
        *ticket = id;
        cv_.notify_all();
        return FRACTAL_OK;
    }

    // FRACTAL_OK and the result once done (the ticket is then forgotten),
    // FRACTAL_E_AGAIN while pending, FRACTAL_E_INVAL for an unknown ticket.
    int poll(uint64_t ticket, fractal_result *res)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end())
            return FRACTAL_E_INVAL;
        if (it->second.state != DONE)
            return FRACTAL_E_AGAIN;
        *res = it->second.res;
        tickets_.erase(it);
        return FRACTAL_OK;
    }

    enum IterOutcome { IDLE, WAITING, RAN };

    // One scheduling iteration: admit from the head of the queue, enqueue
    // the new requests' initialisation, enqueue up to steps_per_iter steps
    // of every active request (longest remaining first), and hand finished
    // requests to retirement.  IDLE: no request queued or active; WAITING:
    // queued requests wait for a slot or arena space held by requests that
    // are retiring.
    IterOutcome iterate()
    {
        std::vector<Admitted> adm;
        std::vector<fractal_request> adm_rq;
        std::vector<ServeIterItem> items;
        int per_iter;
        {
            std::lock_guard<std::mutex> lk(mu_);
            adm = queue_.admit(slot_free_, alloc_);
            const double t = clock_.now();
            for (const Admitted &a : adm) {
                Ticket &tk = tickets_[a.ticket];
                tk.state = ACTIVE;
                tk.res.t_admit = t;
                ServeSlot &sl = slots_[a.slot];
                sl.busy = true;
                sl.ticket = a.ticket;
                sl.offset = a.offset;
                sl.k = tk.rq.k;
                sl.rule = tk.rq.rule;
                sl.steps = tk.rq.steps;
                sl.done = 0;
                sl.alpha = tk.rq.alpha;
                adm_rq.push_back(tk.rq);
            }
            if (adm.empty() && active_count() == 0)
                return queue_.empty() ? IDLE : WAITING;
            per_iter = per_iter_;
        }
        for (size_t q = 0; q < adm.size(); ++q) {
            const int rc = ex_.init_slot(adm[q].slot, slot_copy(adm[q].slot), adm_rq[q]);
            if (rc)
                abort_slots({adm[q].slot}, rc);
        }
        if (!adm.empty()) {
            const int rc = ex_.join_init();
            if (rc) {
                std::vector<int> ids;
                for (const Admitted &a : adm)
                    ids.push_back(a.slot);
                abort_slots(ids, rc);
            }
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (int i = 0; i < (int)slots_.size(); ++i)
                if (slots_[i].busy && slots_[i].done <= slots_[i].steps)
                    items.push_back(ServeIterItem{i, slots_[i], 0});
        }
        if (items.empty())
            return RAN;
        auto rem = [](const ServeSlot &x) { return x.steps - x.done; };
        std::stable_sort(items.begin(), items.end(), [&](const ServeIterItem &a,
                                                         const ServeIterItem &b) {
            return rem(a.s) > rem(b.s);
        });
        const int c = std::min(per_iter, rem(items[0].s));
        if (c > 0) {
            std::vector<ServeIterItem> work;
            for (ServeIterItem &it : items) {
                it.steps = std::min(c, rem(it.s));
                if (it.steps > 0)
                    work.push_back(it);
            }
            const int rc = ex_.run(work);
            if (rc) {
                std::vector<int> ids;
                for (const ServeIterItem &it : items)
                    ids.push_back(it.slot);
                abort_slots(ids, rc);
                return RAN;
            }
        }
        std::vector<std::pair<int, ServeSlot>> fin;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (const ServeIterItem &it : items) {
                ServeSlot &sl = slots_[it.slot];
                sl.done += std::min(c, sl.steps - sl.done);
                if (sl.done >= sl.steps)
                    fin.push_back({it.slot, sl});
            }
            iterations_ += 1;
        }
        for (auto &f : fin) {
            uint64_t token = 0;
            const int rc = ex_.finish(f.first, f.second, &token);
            if (rc) {
                abort_slots({f.first}, rc);
                continue;
            }
            std::lock_guard<std::mutex> lk(mu_);
            slots_[f.first].done = slots_[f.first].steps + 1; // leaves the active set
            tickets_[f.second.ticket].state = RETIRING;
            retire_.push_back(RetireJob{f.second.ticket, f.first, token});
            cv_.notify_all();
        }
        return RAN;
    }

    // Retire the oldest finished request: wait for its last work, copy the
    // result out, stamp it and return its arena range and slot.  False if
    // none is waiting.
    bool retire_one()
    {
        RetireJob job;
        ServeSlot sl;
        void *h_out = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (retire_.empty())
                return false;
            job = retire_.front();
            retire_.pop_front();
            sl = slots_[job.slot];
            h_out = tickets_[job.ticket].rq.h_out;
        }
        uint64_t sum = 0;
        const int rc = ex_.collect(job.token, job.slot, sl, h_out, &sum);
        std::lock_guard<std::mutex> lk(mu_);
        Ticket &tk = tickets_[job.ticket];
        tk.res.status = rc;
        tk.res.checksum = rc ? 0 : sum;
        record_done(tk, sl);
        free_slot(job.slot);
        return true;
    }

    // Latency and throughput of the requests completed so far.
    void stats(fractal_serve_report *st)
    {
        std::lock_guard<std::mutex> lk(mu_);
        std::memset(st, 0, sizeof *st);
        st->submitted = submitted_;
        st->completed = completed_;
        st->failed = failed_;
        st->pending = submitted_ - completed_ - failed_;
        st->iterations = iterations_;
        st->cell_updates = cell_updates_;
        st->t_first_arrival = completed_ ? t_first_arrival_ : 0.0;
        st->t_last_done = completed_ ? t_last_done_ : 0.0;
        if (!lat_.empty()) {
            std::vector<double> v = lat_;
            std::sort(v.begin(), v.end());
            st->p50_latency = nearest_rank(v, 50.0);
            st->p99_latency = nearest_rank(v, 99.0);
            double sum = 0.0;
            for (double x : v)
                sum += x;
            st->mean_latency = sum / (double)v.size();
        }
    }

    // Nearest-rank percentile of a sorted, non-empty sample.
    static double nearest_rank(const std::vector<double> &sorted, double p)
    {
        size_t rank = (size_t)std::ceil(p / 100.0 * (double)sorted.size());
        rank = rank < 1 ? 1 : (rank > sorted.size() ? sorted.size() : rank);
        return sorted[rank - 1];
    }

    // Thread plumbing: the scheduler thread waits here until there may be
    // work (or for `ms` when queued work waits for retirement); the retire
    // thread until a job is queued.  Both return false once stopping and
    // drained.
    bool wait_work(bool waiting, int ms)
    {
        std::unique_lock<std::mutex> lk(mu_);
        if (waiting) {
            // a deadline on the system clock (a short wait: clock steps do
            // not matter), which ThreadSanitizer also understands
            cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(ms));
        } else {
            cv_.wait(lk, [&] { return stopping_ || !queue_.empty() || active_count() > 0; });
        }
        return !(stopping_ && queue_.empty() && active_count() == 0);
    }
    bool wait_retire()
    {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return rstop_ || !retire_.empty(); });
        return !(rstop_ && retire_.empty());
    }
    void stop_scheduling()
    {
        std::lock_guard<std::mutex> lk(mu_);
        stopping_ = true;
        cv_.notify_all();
    }
    void stop_retiring()
    {
        std::lock_guard<std::mutex> lk(mu_);
        rstop_ = true;
        cv_.notify_all();
    }

  private:
    enum TicketState { QUEUED, ACTIVE, RETIRING, DONE };
    struct Ticket {
        fractal_request rq;
        fractal_result res;
        TicketState state;
    };
    struct RetireJob {
        uint64_t ticket = 0;
        int slot = 0;
        uint64_t token = 0;
    };

    int active_count() const
    {
        int c = 0;
        for (const ServeSlot &s : slots_)
            if (s.busy && s.done <= s.steps)
                ++c;
        return c;
    }
    ServeSlot slot_copy(int i)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return slots_[i];
    }

    // Called with mu_ held.
    void free_slot(int i)
    {
        alloc_.release(slots_[i].offset);
        slots_[i] = ServeSlot();
        slot_free_[i] = true;
        cv_.notify_all();
    }

    // Called with mu_ held: stamps and statistics of a finished ticket.
    void record_done(Ticket &tk, const ServeSlot &sl)
    {
        tk.res.t_done = clock_.now();
        tk.state = DONE;
        if (tk.res.status != FRACTAL_OK) {
            ++failed_;
            return;
        }
        ++completed_;
        lat_.push_back(tk.res.t_done - tk.res.t_arrival);
        cell_updates_ += std::pow(3.0, sl.k) * (double)sl.steps;
        if (completed_ == 1 || tk.res.t_arrival < t_first_arrival_)
            t_first_arrival_ = tk.res.t_arrival;
        if (tk.res.t_done > t_last_done_)
            t_last_done_ = tk.res.t_done;
    }

    // Give up on slots after a device error: wait for the device, then fail
    // their tickets with `code` and return their ranges.
    void abort_slots(const std::vector<int> &ids, int code)
    {
        ex_.drain();
        std::lock_guard<std::mutex> lk(mu_);
        for (int i : ids) {
            ServeSlot &s = slots_[i];
            if (!s.busy || s.done > s.steps)
                continue; // already given up, or retiring
            Ticket &tk = tickets_[s.ticket];
            tk.res.status = code;
            record_done(tk, s);
            free_slot(i);
        }
    }

    ServeExecutor &ex_;
    ServeClock &clock_;
    std::mutex mu_;
    std::condition_variable cv_;
    bool stopping_ = false, rstop_ = false;
    int per_iter_;
    uint64_t next_ticket_ = 0;
    std::unordered_map<uint64_t, Ticket> tickets_;
    AdmissionQueue queue_;
    ArenaAllocator alloc_;
    std::vector<ServeSlot> slots_;
    std::vector<bool> slot_free_;
    std::deque<RetireJob> retire_;
    uint64_t submitted_ = 0, completed_ = 0, failed_ = 0, iterations_ = 0;
    double cell_updates_ = 0.0, t_first_arrival_ = 0.0, t_last_done_ = 0.0;
    std::vector<double> lat_;
};

} // namespace fractal
