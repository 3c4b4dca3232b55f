// Host-side admission logic of the serving layer, free of any device code so
// that it can be exercised on the CPU: a first-fit arena over the ciphertext
// budget, the rule that forms batches from the arrival queue, and the
// bookkeeping of every request from submission to completion (including
// cancellation and refusal of requests that exceed the budget).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

#include "ensei.h"

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

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3, kCancelled = 4 };

// What the book keeps per request (times in the caller's clock, seconds).
struct Ticket {
    int shape = -1;
    size_t bytes = 0;      // footprint in the budget
    ReqState state = kQueued;
    int status = ENSEI_OK;
    bool cancel = false;   // cancelled while running: reported as cancelled when its batch ends
    size_t off = 0;        // block in the budget while running
    double t_submit = 0, t_start = 0, t_done = 0;
};

// Request bookkeeping of a server: the queue in arrival order, the arena over
// the budget and the records of every request. Not thread-safe: the server
// calls it under its mutex.
//   submit: refuses (ENSEI_ERR_BUDGET) a request whose footprint exceeds the
//           whole budget, or that would take the bytes waiting in the queue
//           past the queue limit (0 = no limit);
//   cancel: a queued request leaves the queue at once and never takes budget
//           or device time; a running one is marked and, once its batch has
//           finished, released like any other and reported cancelled; a
//           finished request cannot be cancelled (ENSEI_ERR_STATE);
//   admit:  the next batch (next_batch's rule), its requests marked running;
//   finish: a batch has ended with status rc: its blocks return to the arena.
class Book {
   public:
    void reset(size_t budget, size_t queue_limit = 0) {
        arena_.reset(budget);
        queue_.clear();
        recs_.clear();
        queue_limit_ = queue_limit;
        queued_bytes_ = 0;
        peak_used_ = 0;
    }
    void set_queue_limit(size_t bytes) { queue_limit_ = bytes; }
    int submit(uint64_t ticket, int shape, size_t bytes, double now) {
        if (bytes == 0 || recs_.count(ticket)) return ENSEI_ERR_ARG;
        if (align_up(bytes) > arena_.size()) return ENSEI_ERR_BUDGET;
        if (queue_limit_ && queued_bytes_ + align_up(bytes) > queue_limit_) return ENSEI_ERR_BUDGET;
        Ticket t;
        t.shape = shape;
        t.bytes = bytes;
        t.t_submit = now;
        recs_.emplace(ticket, t);
        queue_.push_back(ticket);
        queued_bytes_ += align_up(bytes);
        return ENSEI_OK;
    }
    int cancel(uint64_t ticket, double now) {
        auto it = recs_.find(ticket);
        if (it == recs_.end()) return ENSEI_ERR_ARG;
        Ticket &t = it->second;
        if (t.state == kQueued) {
            queue_.erase(std::find(queue_.begin(), queue_.end(), ticket));
            queued_bytes_ -= align_up(t.bytes);
            t.state = kCancelled;
            t.status = ENSEI_ERR_CANCELLED;
            t.t_done = now;
            return ENSEI_OK;
        }
        if (t.state == kRunning) {
            t.cancel = true;
            return ENSEI_OK;
        }
        return ENSEI_ERR_STATE;
    }
    std::vector<Admitted> admit(int max_batch, double now) {
        auto b = next_batch(queue_, arena_, max_batch, [&](uint64_t k) { return recs_[k].bytes; });
        for (const Admitted &a : b) {
            Ticket &t = recs_[a.ticket];
            t.state = kRunning;
            t.off = a.off;
            t.t_start = now;
            queued_bytes_ -= align_up(t.bytes);
        }
        if (arena_.used() > peak_used_) peak_used_ = arena_.used();
        return b;
    }
    void finish(const std::vector<uint64_t> &tickets, int rc, double now) {
        for (uint64_t k : tickets) {
            Ticket &t = recs_[k];
            arena_.release(t.off, t.bytes);
            t.t_done = now;
            if (t.cancel) {
                t.state = kCancelled;
                t.status = ENSEI_ERR_CANCELLED;
            } else {
                t.state = rc ? kFailed : kDone;
                t.status = rc;
            }
        }
    }
    // Drops a finished record (ENSEI_ERR_ARG if unknown or not finished).
    int forget(uint64_t ticket) {
        auto it = recs_.find(ticket);
        if (it == recs_.end() || it->second.state < kDone) return ENSEI_ERR_ARG;
        recs_.erase(it);
        return ENSEI_OK;
    }
    const Ticket *find(uint64_t ticket) const {
        auto it = recs_.find(ticket);
        return it == recs_.end() ? nullptr : &it->second;
    }
    size_t queued() const { return queue_.size(); }
    size_t queued_bytes() const { return queued_bytes_; }
    size_t used() const { return arena_.used(); }
    size_t peak_used() const { return peak_used_; }
    size_t budget() const { return arena_.size(); }
    const Arena &arena() const { return arena_; }

   private:
    Arena arena_;
    std::deque<uint64_t> queue_;
    std::unordered_map<uint64_t, Ticket> recs_;
    size_t queue_limit_ = 0, queued_bytes_ = 0, peak_used_ = 0;
};

}  // namespace sched
}  // namespace ensei
