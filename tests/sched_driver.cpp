// CPU checks of the serving layer's admission logic (csrc/sched.hpp): the
// first-fit arena, the in-order batch rule, and the request book (refusal of
// over-budget requests, cancellation) driven by a fake executor in place of
// the device. Exits non-zero on a failure.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "sched.hpp"

using namespace ensei::sched;

static int failures = 0;
#define CHECK(cond)                                                \
    do {                                                           \
        if (!(cond)) {                                             \
            printf("FAILED line %d: %s\n", __LINE__, #cond);       \
            ++failures;                                            \
        }                                                          \
    } while (0)

static void arena_basics() {
    Arena a;
    a.reset(10000);
    CHECK(a.size() == 9984);  // whole 256-byte units only
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0);
    CHECK(a.alloc(300, &o2) && o2 == 256);
    CHECK(a.alloc(256, &o3) && o3 == 768);
    CHECK(a.used() == 1024);
    CHECK(!a.alloc(0, &o4));
    CHECK(!a.alloc(9984, &o4));  // does not fit beside the others
    a.release(o2, 300);          // a hole between o1 and o3
    CHECK(a.free_blocks() == 2 && a.largest_free() == 9984 - 1024);
    CHECK(a.alloc(512, &o4) && o4 == 256);  // first fit reuses the hole
    a.release(o4, 512);
    a.release(o1, 100);  // merges with the hole after it
    CHECK(a.free_blocks() == 2);
    a.release(o3, 256);  // merges everything
    CHECK(a.free_blocks() == 1 && a.used() == 0 && a.largest_free() == 9984);
}

static void arena_fragmentation() {
    Arena a;
    a.reset(10 * 1024);
    std::vector<size_t> offs(10);
    for (int i = 0; i < 10; ++i) CHECK(a.alloc(1000, &offs[i]));
    size_t o;
    CHECK(!a.alloc(1, &o));
    for (int i = 0; i < 10; i += 2) a.release(offs[i], 1000);
    CHECK(a.largest_free() == 1024 && a.free_blocks() == 5);
    CHECK(!a.alloc(2000, &o));  // fragmented: no 2 KB run
    for (int i = 1; i < 10; i += 2) a.release(offs[i], 1000);
    CHECK(a.free_blocks() == 1 && a.alloc(10 * 1024, &o) && o == 0);
}

static void batches_in_arrival_order() {
    Arena a;
    a.reset(10 * 1024);
    std::map<uint64_t, size_t> fp = {{1, 4096}, {2, 4096}, {3, 8192}, {4, 1024}, {5, 1024}};
    auto foot = [&](uint64_t t) { return fp[t]; };
    std::deque<uint64_t> q = {1, 2, 3, 4, 5};
    auto b1 = next_batch(q, a, 8, foot);
    // 3 does not fit, and 4, 5 may not overtake it
    CHECK(b1.size() == 2 && b1[0].ticket == 1 && b1[1].ticket == 2);
    CHECK(q.size() == 3 && q.front() == 3);
    a.release(b1[0].off, b1[0].bytes);
    CHECK(next_batch(q, a, 8, foot).empty());  // 4 KB hole + 2 KB tail: still no 8 KB run
    a.release(b1[1].off, b1[1].bytes);
    auto b2 = next_batch(q, a, 8, foot);
    CHECK(b2.size() == 3 && b2[0].ticket == 3 && b2[1].ticket == 4 && b2[2].ticket == 5);
    CHECK(q.empty() && a.used() == 10 * 1024);
}

static void batch_size_limit() {
    Arena a;
    a.reset(1 << 20);
    std::deque<uint64_t> q;
    for (uint64_t t = 1; t <= 10; ++t) q.push_back(t);
    auto foot = [](uint64_t) { return (size_t)1000; };
    CHECK(next_batch(q, a, 4, foot).size() == 4);
    CHECK(next_batch(q, a, 4, foot).size() == 4);
    CHECK(next_batch(q, a, 4, foot).size() == 2);
    CHECK(next_batch(q, a, 4, foot).empty());
}

// Random arrivals and completions: the budget is never exceeded, blocks never
// overlap, admission follows arrival order, and everything is returned.
static void random_stress() {
    std::mt19937_64 g(7);
    Arena a;
    const size_t budget = 64 << 20;
    a.reset(budget);
    std::map<uint64_t, size_t> fp;
    std::deque<uint64_t> q;
    std::vector<Admitted> running;
    uint64_t next = 1, last_admitted = 0;
    for (int step = 0; step < 20000; ++step) {
        if (g() % 3 != 0 && next < 5000) {
            fp[next] = 1 + g() % (12 << 20);
            q.push_back(next++);
        }
        if (!running.empty() && g() % 2 == 0) {
            const size_t k = g() % running.size();
            a.release(running[k].off, running[k].bytes);
            running.erase(running.begin() + k);
        }
        auto b = next_batch(q, a, 1 + (int)(g() % 16), [&](uint64_t t) { return fp[t]; });
        for (const Admitted &x : b) {
            CHECK(x.ticket == last_admitted + 1);
            last_admitted = x.ticket;
            for (const Admitted &y : running) CHECK(x.off + align_up(x.bytes) <= y.off || y.off + align_up(y.bytes) <= x.off);
            CHECK(x.off + align_up(x.bytes) <= budget);
            running.push_back(x);
        }
        CHECK(a.used() <= budget);
    }
    for (const Admitted &x : running) a.release(x.off, x.bytes);
    CHECK(a.used() == 0 && a.free_blocks() == 1);
}

// Refusals at submit: a footprint larger than the whole budget, and bytes
// waiting past the queue limit; nothing is queued for a refused request.
static void book_budget() {
    Book b;
    b.reset(8 * 1024);
    CHECK(b.submit(1, 0, 8 * 1024 + 1, 0.0) == ENSEI_ERR_BUDGET);
    CHECK(b.find(1) == nullptr && b.queued() == 0);
    CHECK(b.submit(1, 0, 8 * 1024, 0.0) == ENSEI_OK);  // exactly the budget fits
    CHECK(b.submit(1, 0, 100, 0.0) == ENSEI_ERR_ARG);   // duplicate ticket
    b.set_queue_limit(10 * 1024);
    CHECK(b.submit(2, 0, 2048, 0.0) == ENSEI_OK);        // 8 KB + 2 KB waiting
    CHECK(b.submit(3, 0, 1, 0.0) == ENSEI_ERR_BUDGET);   // 256 more bytes would pass the cap
    CHECK(b.queued() == 2 && b.queued_bytes() == 10 * 1024);
    auto a = b.admit(8, 1.0);
    CHECK(a.size() == 1 && a[0].ticket == 1 && b.queued_bytes() == 2048);
    CHECK(b.submit(3, 0, 1, 1.0) == ENSEI_OK);           // room in the queue again
}

// Cancellation: a queued request leaves at once and lets the requests behind
// it in; a running one keeps its block until its batch ends and is then
// reported cancelled; a finished one cannot be cancelled.
static void book_cancel() {
    Book b;
    b.reset(10 * 1024);
    CHECK(b.submit(1, 0, 6 * 1024, 0.0) == ENSEI_OK);
    CHECK(b.submit(2, 0, 6 * 1024, 0.0) == ENSEI_OK);  // head of the queue once 1 runs; does not fit beside it
    CHECK(b.submit(3, 0, 1024, 0.0) == ENSEI_OK);
    auto a1 = b.admit(8, 1.0);
    CHECK(a1.size() == 1 && a1[0].ticket == 1);
    CHECK(b.admit(8, 1.0).empty());  // 3 may not overtake 2
    CHECK(b.cancel(2, 2.0) == ENSEI_OK);
    CHECK(b.find(2)->state == kCancelled && b.find(2)->status == ENSEI_ERR_CANCELLED);
    auto a2 = b.admit(8, 2.0);  // 3 goes in beside 1
    CHECK(a2.size() == 1 && a2[0].ticket == 3);
    CHECK(b.cancel(1, 3.0) == ENSEI_OK && b.find(1)->state == kRunning);
    CHECK(b.used() == 7 * 1024);  // 1 still holds its block
    b.finish({1}, ENSEI_OK, 4.0);
    CHECK(b.find(1)->state == kCancelled && b.find(1)->status == ENSEI_ERR_CANCELLED);
    CHECK(b.used() == 1024);
    b.finish({3}, ENSEI_OK, 4.0);
    CHECK(b.find(3)->state == kDone && b.find(3)->status == ENSEI_OK && b.used() == 0);
    CHECK(b.cancel(3, 5.0) == ENSEI_ERR_STATE);
    CHECK(b.cancel(2, 5.0) == ENSEI_ERR_STATE);
    CHECK(b.cancel(99, 5.0) == ENSEI_ERR_ARG);
    CHECK(b.forget(3) == ENSEI_OK && b.find(3) == nullptr && b.forget(3) == ENSEI_ERR_ARG);
    CHECK(b.queued() == 0 && b.queued_bytes() == 0);
}

// A fake executor: every request owns a 64-word output buffer that its batch
// fills with a function of its own inputs only, at completion. Random
// submits, cancels (queued and running), admissions and completions: every
// request that completes holds exactly what it would hold alone, a request
// cancelled while queued is never admitted and its buffer never written,
// the budget is never exceeded, and every block is returned.
static uint64_t fake_result(uint64_t input, int k) {
    uint64_t z = input + 0x9E3779B97F4A7C15ull * (uint64_t)(k + 1);
    z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
    return z ^ (z >> 29);
}

static void book_fake_executor() {
    std::mt19937_64 g(11);
    Book b;
    const size_t budget = 32 << 20;
    b.reset(budget, 200 << 20);
    struct Out {
        uint64_t input;
        std::vector<uint64_t> words;
        bool written = false;
    };
    std::map<uint64_t, Out> outs;
    struct Running {
        std::vector<uint64_t> tickets;
    };
    std::vector<Running> inflight;
    std::map<uint64_t, bool> cancelled_queued;
    uint64_t next = 1;
    int refused = 0, cancels = 0;
    for (int step = 0; step < 20000; ++step) {
        const double now = step;
        if (g() % 2 == 0 && next < 6000) {
            const size_t bytes = 1 + g() % (40 << 20);  // some exceed the 32 MB budget
            const int rc = b.submit(next, 0, bytes, now);
            if (rc == ENSEI_OK) {
                outs[next] = Out{g(), std::vector<uint64_t>(64, 0), false};
            } else {
                CHECK(rc == ENSEI_ERR_BUDGET);
                CHECK(bytes > budget || b.queued_bytes() + align_up(bytes) > (200u << 20));
                ++refused;
            }
            ++next;
        }
        if (g() % 7 == 0 && next > 1) {
            const uint64_t t = 1 + g() % (next - 1);
            const Ticket *k = b.find(t);
            if (k) {
                const bool queued = k->state == kQueued;
                const int rc = b.cancel(t, now);
                if (k->state >= kDone && !queued && rc == ENSEI_ERR_STATE) {
                } else {
                    CHECK(rc == ENSEI_OK);
                    ++cancels;
                    if (queued) cancelled_queued[t] = true;
                }
            }
        }
        if (!inflight.empty() && g() % 3 == 0) {
            const size_t i = g() % inflight.size();
            for (uint64_t t : inflight[i].tickets) {  // the "device" writes each request's own output
                Out &o = outs[t];
                for (int k = 0; k < 64; ++k) o.words[k] = fake_result(o.input, k);
                o.written = true;
            }
            b.finish(inflight[i].tickets, ENSEI_OK, now);
            inflight.erase(inflight.begin() + i);
        }
        auto a = b.admit(1 + (int)(g() % 8), now);
        if (!a.empty()) {
            Running r;
            for (const Admitted &x : a) {
                CHECK(!cancelled_queued.count(x.ticket));
                CHECK(x.off + align_up(x.bytes) <= budget);
                r.tickets.push_back(x.ticket);
            }
            inflight.push_back(r);
        }
        CHECK(b.used() <= budget);
    }
    for (auto &r : inflight) {
        for (uint64_t t : r.tickets) {
            Out &o = outs[t];
            for (int k = 0; k < 64; ++k) o.words[k] = fake_result(o.input, k);
            o.written = true;
        }
        b.finish(r.tickets, ENSEI_OK, 1e9);
    }
    while (b.queued()) {  // drain what is left, one batch at a time
        auto a = b.admit(16, 2e9);
        CHECK(!a.empty());
        std::vector<uint64_t> ts;
        for (const Admitted &x : a) {
            Out &o = outs[x.ticket];
            for (int k = 0; k < 64; ++k) o.words[k] = fake_result(o.input, k);
            o.written = true;
            ts.push_back(x.ticket);
        }
        b.finish(ts, ENSEI_OK, 2e9);
    }
    int done = 0;
    for (auto &kv : outs) {
        const Ticket *k = b.find(kv.first);
        CHECK(k != nullptr && k->state >= kDone);
        if (cancelled_queued.count(kv.first)) {
            CHECK(k->state == kCancelled && !kv.second.written);
            continue;
        }
        if (k->state == kDone) {
            ++done;
            for (int i = 0; i < 64; ++i) CHECK(kv.second.words[i] == fake_result(kv.second.input, i));
        } else {
            CHECK(k->state == kCancelled);  // cancelled while running: ran, reported cancelled
        }
    }
    CHECK(b.used() == 0 && b.arena().free_blocks() == 1 && b.queued_bytes() == 0);
    CHECK(refused > 0 && cancels > 0 && done > 1000);
}

int main() {
    arena_basics();
    arena_fragmentation();
    batches_in_arrival_order();
    batch_size_limit();
    random_stress();
    book_budget();
    book_cancel();
    book_fake_executor();
    printf("%s\n", failures ? "sched checks FAILED" : "sched checks ok");
    return failures ? 1 : 0;
}
