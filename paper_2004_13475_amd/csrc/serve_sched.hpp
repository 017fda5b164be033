// serve_sched.hpp -- host-only scheduling pieces of the request server:
// a first-fit arena allocator with coalescing and a FIFO admission queue.
// No HIP here, so the logic is unit-tested on the CPU with a plain compiler.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

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

} // namespace fractal
