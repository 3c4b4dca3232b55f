// CPU checks of the serving layer's admission logic (csrc/sched.hpp): the
// first-fit arena and the in-order batch rule. Exits non-zero on a failure.
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

int main() {
    arena_basics();
    arena_fragmentation();
    batches_in_arrival_order();
    batch_size_limit();
    random_stress();
    printf("%s\n", failures ? "sched checks FAILED" : "sched checks ok");
    return failures ? 1 : 0;
}
