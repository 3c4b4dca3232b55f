// Host-side admission logic of the serving layer, free of any device code so
// that it can be exercised on the CPU: a first-fit arena over the ciphertext
// budget and the rule that forms batches from the arrival queue.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace ensei {
namespace sched {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) in 256-byte units, with coalescing of
// free neighbours. Offsets are relative to the start of the budget.
class Arena {
   public:
    void reset(size_t size) {
        free_.clear();
        size = size / kAlign * kAlign;
        if (size) free_[0] = size;
        used_ = 0;
        size_ = size;
    }
    bool alloc(size_t n, size_t *off) {
        n = align_up(n);
        if (n == 0) return false;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align_up(n);
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

   private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t used_ = 0, size_ = 0;
};

// One admitted request: its ticket and its block of the budget.
struct Admitted {
    uint64_t ticket;
    size_t off, bytes;
};

// Forms the next batch: requests leave the queue strictly in arrival order
// while their footprint fits the arena (the head of the queue waits for
// space rather than being overtaken), at most max_batch of them. footprint
// maps a ticket to its bytes. Returns an empty batch if the head does not fit.
template <class Footprint>
std::vector<Admitted> next_batch(std::deque<uint64_t> &queue, Arena &arena, int max_batch, Footprint footprint) {
    std::vector<Admitted> batch;
    while (!queue.empty() && (int)batch.size() < max_batch) {
        const uint64_t t = queue.front();
        const size_t bytes = footprint(t);
        size_t off;
        if (!arena.alloc(bytes, &off)) break;
        batch.push_back(Admitted{t, off, bytes});
        queue.pop_front();
    }
    return batch;
}

}  // namespace sched
}  // namespace ensei
