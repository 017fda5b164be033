// CPU test of the request server's scheduler core (ServeCore) with a fake
// executor and a fake clock: budget enforcement, FIFO admission without
// skip-ahead, slot reuse, iterations of at most steps_per_iter steps,
// p50/p99 bookkeeping, and a failing executor failing exactly the requests
// it touched.  Built with g++ and sanitizers by test_host_api.py; also run
// with the core's two threads against the fake executor.
#include <cassert>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../paper_2004_13475_amd/csrc/serve_sched.hpp"

using namespace fractal;

struct FakeClock : ServeClock {
    double t = 100.0;
    double now() override { return t; }
};

// Records every call; `fail_run_at` makes the n-th run() fail (1-based),
// `fail_init_ticket` makes init_slot fail for one ticket's slot.
struct FakeExecutor : ServeExecutor {
    size_t cap;
    int runs = 0, fail_run_at = -1;
    uint64_t fail_init_ticket = 0;
    std::vector<std::vector<ServeIterItem>> run_log;
    std::map<uint64_t, int> steps_seen; // ticket -> steps enqueued
    std::vector<uint64_t> init_order;
    std::mutex token_mu; // finish() and collect() run on different threads
    std::set<uint64_t> live_tokens;
    uint64_t next_token = 1;
    int drains = 0;
    explicit FakeExecutor(size_t c) : cap(c) {}
    size_t state_capacity() const override { return cap; }
    int init_slot(int, const ServeSlot &s, const fractal_request &) override
    {
        init_order.push_back(s.ticket);
        assert(s.offset + serve_footprint(s.k, s.rule) <= cap);
        return s.ticket == fail_init_ticket ? FRACTAL_E_DEVICE : FRACTAL_OK;
    }
    int join_init() override { return FRACTAL_OK; }
    int run(const std::vector<ServeIterItem> &items) override
    {
        ++runs;
        run_log.push_back(items);
        if (runs == fail_run_at)
            return FRACTAL_E_DEVICE;
        for (const ServeIterItem &it : items) {
            assert(it.steps > 0 && it.s.done + it.steps <= it.s.steps);
            assert(steps_seen[it.s.ticket] == it.s.done); // steps continue where they stopped
            steps_seen[it.s.ticket] += it.steps;
        }
        return FRACTAL_OK;
    }
    int finish(int, const ServeSlot &s, uint64_t *token) override
    {
        assert(steps_seen[s.ticket] == s.steps);
        std::lock_guard<std::mutex> lk(token_mu);
        *token = next_token++;
        live_tokens.insert(*token);
        return FRACTAL_OK;
    }
    int collect(uint64_t token, int, const ServeSlot &s, void *, uint64_t *sum) override
    {
        {
            std::lock_guard<std::mutex> lk(token_mu);
            assert(live_tokens.erase(token) == 1);
        }
        *sum = (uint64_t)s.k * 1000u + (uint64_t)s.steps; // a value the test can predict
        return FRACTAL_OK;
    }
    void drain() override { ++drains; }
};

static fractal_request req(int k, int rule, int steps, double t_arrival = -1.0)
{
    fractal_request r;
    std::memset(&r, 0, sizeof r);
    r.k = k;
    r.rule = rule;
    r.steps = steps;
    r.alpha = 0.2f;
    r.t_arrival = t_arrival;
    return r;
}

static uint64_t submit(ServeCore &c, const fractal_request &r)
{
    uint64_t t = 0;
    const char *msg;
    const int rc = c.submit(r, &t, &msg);
    assert(rc == FRACTAL_OK);
    return t;
}

static void drain_all(ServeCore &c, int max_iter = 10000)
{
    for (int i = 0; i < max_iter; ++i) {
        const auto o = c.iterate();
        while (c.retire_one()) {
        }
        if (o == ServeCore::IDLE)
            return;
    }
    assert(!"scheduler did not drain");
}

static void test_validation()
{
    FakeExecutor ex(serve_footprint(8, FRACTAL_RULE_HEAT));
    FakeClock clk;
    ServeCore c(ex, clk, 2, 16);
    uint64_t t;
    const char *msg;
    assert(c.submit(req(9, FRACTAL_RULE_HEAT, 5), &t, &msg) == FRACTAL_E_NOMEM);
    assert(c.submit(req(17, 0, 5), &t, &msg) == FRACTAL_E_INVAL);
    assert(c.submit(req(5, 2, 5), &t, &msg) == FRACTAL_E_INVAL);
    assert(c.submit(req(5, 0, -1), &t, &msg) == FRACTAL_E_INVAL);
    fractal_request bad = req(5, FRACTAL_RULE_HEAT, 5);
    bad.alpha = 0.3f;
    assert(c.submit(bad, &t, &msg) == FRACTAL_E_INVAL);
    bad.alpha = std::nanf("");
    assert(c.submit(bad, &t, &msg) == FRACTAL_E_INVAL);
    fractal_result res;
    assert(c.poll(12345, &res) == FRACTAL_E_INVAL);
    // one that fits exactly is accepted
    t = submit(c, req(8, FRACTAL_RULE_HEAT, 3));
    assert(c.poll(t, &res) == FRACTAL_E_AGAIN);
    drain_all(c);
    assert(c.poll(t, &res) == FRACTAL_OK && res.status == FRACTAL_OK);
    assert(res.checksum == 8003u);
    assert(c.poll(t, &res) == FRACTAL_E_INVAL); // forgotten once polled
}

// Budget: room for two requests of level 10 (uint8); the third waits until
// one retires, then takes the freed range; arena use never exceeds the budget.
static void test_budget_and_slot_reuse()
{
    const size_t one = serve_footprint(10, FRACTAL_RULE_CA);
    FakeExecutor ex(2 * one);
    FakeClock clk;
    ServeCore c(ex, clk, 4, 16);
    const uint64_t a = submit(c, req(10, 0, 20));
    const uint64_t b = submit(c, req(10, 0, 40));
    const uint64_t d = submit(c, req(10, 0, 10));
    assert(c.iterate() == ServeCore::RAN);
    assert(ex.init_order.size() == 2 && ex.init_order[0] == a && ex.init_order[1] == b);
    assert(ex.run_log.back().size() == 2);
    assert(c.iterate() == ServeCore::RAN); // a finishes its 20 steps (16 + 4)
    assert(ex.init_order.size() == 2);     // d still waits: a has not retired
    assert(c.retire_one());
    assert(!c.retire_one());
    assert(c.iterate() == ServeCore::RAN); // d admitted into a's range and slot 0
    assert(ex.init_order.size() == 3 && ex.init_order[2] == d);
    assert(ex.run_log.back().size() == 2);
    bool d_in_slot0 = false;
    for (const ServeIterItem &it : ex.run_log.back())
        if (it.s.ticket == d)
            d_in_slot0 = it.slot == 0 && it.s.offset == 0;
    assert(d_in_slot0);
    drain_all(c);
    fractal_result r;
    for (uint64_t t : {a, b, d}) {
        assert(c.poll(t, &r) == FRACTAL_OK);
        assert(r.status == FRACTAL_OK && r.t_arrival <= r.t_admit && r.t_admit <= r.t_done);
    }
    fractal_serve_report st;
    c.stats(&st);
    assert(st.submitted == 3 && st.completed == 3 && st.failed == 0 && st.pending == 0);
    assert(st.cell_updates == std::pow(3.0, 10) * 70.0);
}

// FIFO without skip-ahead: a large request at the head blocks smaller later
// ones while it does not fit.
static void test_fifo_no_skip_ahead()
{
    const size_t small = serve_footprint(8, FRACTAL_RULE_CA);
    const size_t big = serve_footprint(10, FRACTAL_RULE_HEAT);
    FakeExecutor ex(big + small / 2); // s1 resident leaves less than big
    FakeClock clk;
    ServeCore c(ex, clk, 8, 16);
    const uint64_t s1 = submit(c, req(8, 0, 50));
    const uint64_t b1 = submit(c, req(10, 1, 5));  // fits only once s1 leaves
    const uint64_t s2 = submit(c, req(8, 0, 5));   // would fit now, must wait
    c.iterate();
    assert(ex.init_order.size() == 1 && ex.init_order[0] == s1);
    for (int i = 0; i < 3; ++i) {
        c.iterate();
        assert(ex.init_order.size() == 1); // nothing overtakes b1
    }
    while (!c.retire_one())
        c.iterate();
    c.iterate();
    assert(ex.init_order.size() == 2 && ex.init_order[1] == b1); // s2 still does not fit
    drain_all(c);
    assert(ex.init_order.size() == 3 && ex.init_order[2] == s2);
}

// Iterations of at most steps_per_iter steps per request, longest remaining
// first; a request of zero steps finishes in its first iteration.
static void test_iterations()
{
    FakeExecutor ex(serve_footprint(12, 1) * 4);
    FakeClock clk;
    ServeCore c(ex, clk, 4, 16);
    const uint64_t a = submit(c, req(9, 1, 37));
    const uint64_t z = submit(c, req(9, 0, 0));
    c.set_steps_per_iter(10);
    drain_all(c);
    // 37 steps in iterations of 10, 10, 10, 7; the zero-step request is
    // never part of a launch
    std::vector<int> seen;
    for (const auto &it : ex.run_log) {
        assert(it.size() == 1 && it[0].s.ticket == a);
        seen.push_back(it[0].steps);
    }
    assert((seen == std::vector<int>{10, 10, 10, 7}));
    fractal_result r;
    assert(c.poll(z, &r) == FRACTAL_OK && r.status == FRACTAL_OK && r.checksum == 9000u);
}

// Latency percentiles are nearest-rank over completed requests: with
// latencies 1..100 (fake clock), p50 = 50 and p99 = 99.
static void test_latency_bookkeeping()
{
    FakeExecutor ex(serve_footprint(6, 0) * 200);
    FakeClock clk;
    ServeCore c(ex, clk, 1, 16); // one slot: requests run one after another
    std::vector<uint64_t> ts;
    for (int i = 0; i < 100; ++i)
        ts.push_back(submit(c, req(6, 0, 1, 0.0)));
    for (int i = 0; i < 100; ++i) {
        clk.t = (double)(i + 1); // request i completes at t = i + 1
        c.iterate();
        assert(c.retire_one());
    }
    fractal_serve_report st;
    c.stats(&st);
    assert(st.completed == 100 && st.pending == 0);
    assert(st.p50_latency == 50.0 && st.p99_latency == 99.0);
    assert(std::fabs(st.mean_latency - 50.5) < 1e-12);
    assert(st.t_first_arrival == 0.0 && st.t_last_done == 100.0);
    std::vector<double> one{7.0};
    assert(ServeCore::nearest_rank(one, 99.0) == 7.0);
}

// A device failure in an iteration fails exactly the requests of that
// iteration with E_DEVICE and returns their ranges; requests admitted later
// complete; a failing initialisation fails only its own request.
static void test_failures()
{
    const size_t one = serve_footprint(9, 0);
    FakeExecutor ex(3 * one);
    FakeClock clk;
    ServeCore c(ex, clk, 3, 4);
    ex.fail_run_at = 2;
    const uint64_t a = submit(c, req(9, 0, 12));
    const uint64_t b = submit(c, req(9, 0, 2));
    c.iterate();                           // run 1: a 4, b 2 (b finishes)
    c.iterate();                           // run 2 fails: only a is active
    const uint64_t d = submit(c, req(9, 0, 6));
    ex.fail_init_ticket = submit(c, req(9, 0, 3));
    drain_all(c);
    fractal_result r;
    assert(c.poll(a, &r) == FRACTAL_OK && r.status == FRACTAL_E_DEVICE);
    assert(c.poll(b, &r) == FRACTAL_OK && r.status == FRACTAL_OK);
    assert(c.poll(d, &r) == FRACTAL_OK && r.status == FRACTAL_OK && r.checksum == 9006u);
    assert(c.poll(ex.fail_init_ticket, &r) == FRACTAL_OK && r.status == FRACTAL_E_DEVICE);
    assert(ex.drains >= 2 && ex.live_tokens.empty());
    fractal_serve_report st;
    c.stats(&st);
    assert(st.completed == 2 && st.failed == 2 && st.pending == 0);
}

// The two threads the server runs, against the fake executor: every ticket
// completes, in any interleaving.
static void test_threads()
{
    FakeExecutor ex(serve_footprint(8, 1) * 3);
    FakeClock clk;
    ServeCore c(ex, clk, 2, 8);
    std::thread worker([&] {
        bool waiting = false;
        while (c.wait_work(waiting, 1))
            waiting = c.iterate() == ServeCore::WAITING;
    });
    std::thread retirer([&] {
        while (c.wait_retire())
            (void)c.retire_one();
    });
    std::vector<uint64_t> ts;
    for (int i = 0; i < 200; ++i)
        ts.push_back(submit(c, req(4 + i % 5, i % 2, i % 23)));
    c.stop_scheduling();
    worker.join();
    c.stop_retiring();
    retirer.join();
    fractal_result r;
    for (uint64_t t : ts)
        assert(c.poll(t, &r) == FRACTAL_OK && r.status == FRACTAL_OK);
    const char *msg;
    uint64_t t;
    assert(c.submit(req(5, 0, 1), &t, &msg) == FRACTAL_E_INVAL); // shut down
}

int main(int argc, char **argv)
{
    if (argc > 1 && std::string(argv[1]) == "threads") { // the threaded test alone
        test_threads();
        std::puts("serve_core threads ok");
        return 0;
    }
    test_validation();
    test_budget_and_slot_reuse();
    test_fifo_no_skip_ahead();
    test_iterations();
    test_latency_bookkeeping();
    test_failures();
    test_threads();
    std::puts("serve_core ok");
    return 0;
}
