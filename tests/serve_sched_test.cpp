// CPU unit test of the request server's scheduling pieces (arena allocator,
// FIFO admission).  Built with g++ and sanitizers by test_host_api.py.
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2004_13475_amd/csrc/serve_sched.hpp"

using namespace fractal;

static void test_allocator_basic()
{
    ArenaAllocator a(1 << 20, 256);
    size_t o1, o2, o3;
    assert(a.alloc(1000, &o1) && o1 == 0);
    assert(a.alloc(256, &o2) && o2 == 1024);
    assert(a.alloc(1, &o3) && o3 == 1280);
    assert(a.in_use() == 1024 + 256 + 256);
    assert(a.release(o2));
    assert(!a.release(o2)); // double free is refused
    size_t o4;
    assert(a.alloc(200, &o4) && o4 == 1024); // first fit reuses the hole
    assert(a.release(o1) && a.release(o3) && a.release(o4));
    assert(a.in_use() == 0 && a.free_ranges() == 1 && a.largest_free() == (1u << 20));
    size_t big;
    assert(!a.alloc((1 << 20) + 1, &big));
    assert(!a.fits_ever((1 << 20) + 1) && a.fits_ever(1 << 20));
}

static void test_allocator_random_coalesce()
{
    std::mt19937_64 rng(2004);
    ArenaAllocator a(64 << 20, 256);
    std::vector<size_t> live;
    for (int it = 0; it < 20000; ++it) {
        if (!live.empty() && (rng() % 2 == 0)) {
            size_t i = rng() % live.size();
            assert(a.release(live[i]));
            live.erase(live.begin() + (long)i);
        } else {
            size_t off;
            size_t sz = 1 + rng() % (1 << 20);
            if (a.alloc(sz, &off)) {
                assert(off % 256 == 0 && off + a.round(sz) <= a.capacity());
                live.push_back(off);
            }
        }
    }
    for (size_t o : live)
        assert(a.release(o));
    assert(a.in_use() == 0 && a.free_ranges() == 1);
}

static void test_admission_fifo_and_budget()
{
    ArenaAllocator a(1000 * 256, 256);
    AdmissionQueue q;
    std::vector<bool> slots(2, true);
    q.push(1, 600 * 256); // fits
    q.push(2, 600 * 256); // does not fit while 1 is resident
    q.push(3, 10 * 256);  // would fit, but must not overtake 2
    auto adm = q.admit(slots, a);
    assert(adm.size() == 1 && adm[0].ticket == 1 && adm[0].slot == 0);
    adm = q.admit(slots, a);
    assert(adm.empty() && q.size() == 2); // head-of-line: no skip-ahead
    a.release(0);
    slots[0] = true;
    adm = q.admit(slots, a);
    assert(adm.size() == 2 && adm[0].ticket == 2 && adm[1].ticket == 3);
    assert(adm[0].slot == 0 && adm[1].slot == 1);
    q.push(4, 1);
    adm = q.admit(slots, a); // no free slot
    assert(adm.empty() && q.size() == 1);
}

int main()
{
    test_allocator_basic();
    test_allocator_random_coalesce();
    test_admission_fifo_and_budget();
    std::puts("serve_sched ok");
    return 0;
}
