// Serving: continuous batching of secure-convolution requests of mixed shapes.
//
// A worker thread owns the device work. Each round it admits queued requests
// in arrival order while their ciphertext footprint (x^, ct_in, ct_out, m)
// fits the free part of the budget (an arena carved out of one allocation),
// groups the admitted requests into a batch, and enqueues the batch on one of
// a few HIP streams: per request NTT2D and Enc, one persistent HomConv launch
// over the tiles of every request of the batch, then per request Dec, the
// client's INTT2D and the server's share. Batches on different streams
// overlap on the device. When a batch's completion event has fired its arena
// blocks are released and queued requests are admitted into the space.
// Ciphertexts never leave the device between Enc, HomConv and Dec.
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ensei_internal.hpp"
#include "sched.hpp"

namespace ensei {
namespace {

using Clock = std::chrono::steady_clock;

using sched::Arena;
using sched::Book;
using sched::kAlign;

struct Shape {
    ensei_shape d;
    int64_t F;
    uint32_t *w_hat = nullptr;
    int8_t *w_pack = nullptr;
    size_t wpack_bytes = 0;
    size_t footprint = 0;  // arena bytes of one request
    bool narrow = false;   // HomConv on the narrow-input kernel (folded fragments), outside the shared launch
};

// A submitted request's buffers until it is admitted (or cancelled), and the
// event that marks its inputs complete on the caller's stream.
struct Pending {
    ensei_request io;
    hipEvent_t ready = nullptr;
};

// One admitted request, copied out of the shared state so that the batch can
// be enqueued without holding the server's lock.
struct Job {
    uint64_t ticket;
    Shape sh;
    ensei_request io;
    hipEvent_t ready;
    size_t off;
    hipEvent_t done = nullptr;  // recorded after the request's last kernel
    bool finished = false;
};

struct Batch {
    std::vector<Job> jobs;
    hipStream_t stream;
    int slot;  // launch-table slot, busy until every job of the batch has finished
    int remaining = 0;
};

}  // namespace
}  // namespace ensei

using namespace ensei;

struct ensei_server {
    ensei_ctx *ctx = nullptr;
    size_t budget = 0;
    int nstreams = 0, max_batch = 0;
    uint8_t *pool = nullptr;
    std::deque<Shape> shapes;  // grows under mu; elements never move
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    // launch tables of the multi-problem HomConv: per slot max_batch entries,
    // device copy and pinned host staging; a slot is busy while its batch runs
    HcLayer *d_tables = nullptr, *h_tables = nullptr;
    std::vector<int> free_slots;
    std::vector<hipEvent_t> event_pool;  // request completion
    std::vector<hipEvent_t> ready_pool;  // callers' input streams

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    Book book;
    std::unordered_map<uint64_t, Pending> pending;
    std::deque<Batch> inflight;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    Clock::time_point t0 = Clock::now();
    uint64_t n_done = 0, n_failed = 0, n_batches = 0, n_cancelled = 0, n_refused = 0;
    // seeded ciphertexts (ensei_server_create_seeded): a request keeps only
    // the b words of its input ciphertexts
    bool seeded = false;
};

namespace ensei {
namespace {

double secs(const ensei_server *S, Clock::time_point t) { return std::chrono::duration<double>(t - S->t0).count(); }
double now_s(const ensei_server *S) { return secs(S, Clock::now()); }

// Arena layout of one request: x^ [Cin][F] u32, ct_in [F][n+1][Cin] u64
// (seeded: the b words, [F][Cin]), ct_out [F][n+1][Cout] u64, m [Cout][F] u32
// (each 256-byte aligned).
struct Parts {
    size_t x_hat, ct_in, ct_out, m, total;
};
Parts parts_of(const ensei_shape &d, bool seeded = false) {
    auto al = [](size_t v) { return (v + kAlign - 1) / kAlign * kAlign; };
    const size_t F = (size_t)d.H * d.W;
    Parts p;
    p.x_hat = 0;
    p.ct_in = al(F * d.Cin * 4);
    p.ct_out = p.ct_in + al(F * (seeded ? 1 : d.n + 1) * d.Cin * 8);
    p.m = p.ct_out + al(F * (d.n + 1) * d.Cout * 8);
    p.total = p.m + al(F * d.Cout * 4);
    return p;
}

// Enqueues one batch. Called WITHOUT the server's lock: it reads only the
// batch's own jobs, its launch-table slot and the arena memory of its
// requests. The jobs keep their arrival order, and each request's completion
// event follows its own last kernel, so that a request does not wait for the
// decryption of the requests after it. Returns a status; on error nothing of
// the batch is left running once its stream has been synchronised.
int launch_batch(ensei_server *S, Batch &b) {
    const hipStream_t st = b.stream;
    HcLayer *tab = S->h_tables + (size_t)b.slot * S->max_batch;
    int np = 0;
    int64_t tile0 = 0;
    int rc = ENSEI_OK;
    // inputs produced by pending work on the callers' streams
    for (const Job &j : b.jobs)
        if (j.ready && hipStreamWaitEvent(st, j.ready, 0) != hipSuccess) return ENSEI_ERR_HIP;
    for (const Job &j : b.jobs) {
        const Shape &sh = j.sh;
        const ensei_shape &d = sh.d;
        const Parts pt = parts_of(d, S->seeded);
        uint8_t *base = S->pool + j.off;
        uint32_t *x_hat = reinterpret_cast<uint32_t *>(base + pt.x_hat);
        uint64_t *ct_in = reinterpret_cast<uint64_t *>(base + pt.ct_in);
        uint64_t *ct_out = reinterpret_cast<uint64_t *>(base + pt.ct_out);
        rc = ensei_ntt2d(S->ctx, j.io.x, x_hat, d.Cin, d.H, d.W, st);
        if (!rc)
            rc = S->seeded ? ensei_encrypt_seeded(S->ctx, x_hat, j.io.s, j.io.e, 1, d.Cin, sh.F, d.n, j.io.seed_a, 0,
                                                  ct_in, st)
                           : ensei_encrypt(S->ctx, x_hat, j.io.s, j.io.e, 1, d.Cin, sh.F, d.n, j.io.seed_a, 0, ct_in, st);
        HcLayer h;
        if (!rc)
            rc = homconv_problem(S->ctx, &h, ct_in, sh.w_pack, j.io.r, 1, d.Cin, d.Cout, sh.F, d.n, ct_out,
                                 sh.wpack_bytes, S->seeded);
        h.seed_a = S->seeded ? j.io.seed_a : 0;
        h.idx0 = 0;
        // narrow and deep shapes run on their own kernels, the others share one launch
        const bool alone = !rc && (sh.narrow || homconv_deep_fits(h, S->seeded));
        if (alone) rc = homconv_launch(S->ctx, &h, nullptr, 1, !sh.narrow, HcSchedule{0, 0}, st, S->seeded);
        if (rc) break;
        if (alone) continue;
        h.n_items = frag_items(d.Cin, true);
        h.tile0 = tile0;
        tile0 += h.n_tiles;
        tab[np++] = h;
    }
    if (!rc && np > 1) {
        HcLayer *dtab = S->d_tables + (size_t)b.slot * S->max_batch;
        if (hipMemcpyAsync(dtab, tab, np * sizeof(HcLayer), hipMemcpyHostToDevice, st) != hipSuccess)
            rc = ENSEI_ERR_HIP;
        if (!rc) rc = homconv_launch(S->ctx, tab, dtab, np, true, HcSchedule{0, 0}, st, S->seeded);
    } else if (!rc && np == 1) {
        rc = homconv_launch(S->ctx, tab, nullptr, 1, true, HcSchedule{0, 0}, st, S->seeded);
    }
    for (Job &j : b.jobs) {
        if (rc) break;
        const Shape &sh = j.sh;
        const ensei_shape &d = sh.d;
        const Parts pt = parts_of(d, S->seeded);
        uint8_t *base = S->pool + j.off;
        const uint64_t *ct_out = reinterpret_cast<const uint64_t *>(base + pt.ct_out);
        uint32_t *m = reinterpret_cast<uint32_t *>(base + pt.m);
        rc = ensei_decrypt(S->ctx, ct_out, j.io.s, 1, d.Cout, sh.F, d.n, m, st);
        if (!rc) rc = ensei_intt2d(S->ctx, m, j.io.s_a, d.Cout, d.H, d.W, st);
        if (!rc) rc = ensei_server_share(S->ctx, j.io.r, j.io.s_b, d.Cout, d.H, d.W, st);
        if (!rc && hipEventRecord(j.done, st) != hipSuccess) rc = ENSEI_ERR_HIP;
    }
    return rc;
}

// One request of a batch has ended (caller holds the lock): the book releases
// its budget and records the outcome; its events return to their pools.
void finish_job(ensei_server *S, Batch &b, Job &j, int rc) {
    if (j.finished) return;
    j.finished = true;
    --b.remaining;
    S->book.finish({j.ticket}, rc, now_s(S));
    const sched::Ticket *k = S->book.find(j.ticket);
    if (k->state == sched::kDone)
        ++S->n_done;
    else if (k->state == sched::kFailed)
        ++S->n_failed;
    if (j.ready) S->ready_pool.push_back(j.ready);
    S->event_pool.push_back(j.done);
}

// Every request of the batch has ended: its launch-table slot is free again.
void finish_batch(ensei_server *S, Batch &b, int rc) {
    for (Job &j : b.jobs) finish_job(S, b, j, rc);
    S->free_slots.push_back(b.slot);
}

void worker_loop(ensei_server *S) {
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        // retire finished requests, and batches whose requests have all ended
        for (auto it = S->inflight.begin(); it != S->inflight.end();) {
            bool any = false;
            for (Job &j : it->jobs) {
                if (j.finished) continue;
                const hipError_t q = hipEventQuery(j.done);
                if (q == hipErrorNotReady) break;  // later jobs of the stream come after it
                finish_job(S, *it, j, q == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP);
                any = true;
            }
            if (any) S->cv_done.notify_all();
            if (it->remaining == 0) {
                S->free_slots.push_back(it->slot);
                it = S->inflight.erase(it);
            } else {
                ++it;
            }
        }
        // admit queued requests in arrival order while they fit, one batch
        // per free launch slot
        while (S->book.queued() && !S->free_slots.empty()) {
            const auto admitted = S->book.admit(S->max_batch, now_s(S));
            if (admitted.empty()) break;
            Batch b;
            for (const sched::Admitted &a : admitted) {
                auto pit = S->pending.find(a.ticket);
                const int shape = S->book.find(a.ticket)->shape;
                Job j{a.ticket, S->shapes[shape], pit->second.io, pit->second.ready, a.off};
                j.done = S->event_pool.back();
                S->event_pool.pop_back();
                b.jobs.push_back(j);
                S->pending.erase(pit);
            }
            b.remaining = (int)b.jobs.size();
            b.slot = S->free_slots.back();
            S->free_slots.pop_back();
            b.stream = S->streams[S->next_stream];
            S->next_stream = (S->next_stream + 1) % S->nstreams;
            ++S->n_batches;
            // enqueue without the lock, so that submits, polls and cancels
            // are not held up by the launches
            lk.unlock();
            const int rc = launch_batch(S, b);
            if (rc) (void)hipStreamSynchronize(b.stream);  // enqueued work must end before the memory is reused
            lk.lock();
            if (rc) {
                finish_batch(S, b, rc);
                S->cv_done.notify_all();
            } else {
                S->inflight.push_back(std::move(b));
            }
        }
        if (S->stop && !S->book.queued() && S->inflight.empty()) break;
        if (S->inflight.empty() && (!S->book.queued() || S->free_slots.empty()) && !S->stop) {
            S->cv_work.wait(lk);
        } else {
            // device work pending: poll its events at a fine interval
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

void destroy(ensei_server *S) {
    if (S->worker.joinable()) {
        {
            std::lock_guard<std::mutex> g(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->worker.join();
    }
    for (hipStream_t s : S->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : S->ready_pool) (void)hipEventDestroy(e);
    for (auto &kv : S->pending)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (Shape &sh : S->shapes) {
        if (sh.w_hat) (void)hipFree(sh.w_hat);
        if (sh.w_pack) (void)hipFree(sh.w_pack);
    }
    if (S->pool) (void)hipFree(S->pool);
    if (S->d_tables) (void)hipFree(S->d_tables);
    if (S->h_tables) (void)hipHostFree(S->h_tables);
    delete S;
}

}  // namespace
}  // namespace ensei

extern "C" {

size_t ensei_request_bytes(const ensei_shape *shape) {
    if (!shape || shape->H <= 0 || shape->W <= 0 || shape->Cin <= 0 || shape->Cout <= 0 || shape->n <= 0) return 0;
    return parts_of(*shape).total;
}

static int server_create(ensei_ctx *ctx, size_t budget_bytes, int nstreams, int max_batch, ensei_server **out,
                         bool seeded) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out || budget_bytes == 0 || nstreams < 1 || nstreams > 8 || max_batch < 1 || max_batch > 256)
        return ENSEI_ERR_ARG;
    *out = nullptr;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    ensei_server *S = new ensei_server;
    S->ctx = ctx;
    S->seeded = seeded;
    S->budget = (budget_bytes + kAlign - 1) / kAlign * kAlign;
    S->nstreams = nstreams;
    S->max_batch = max_batch;
    const int slots = 2 * nstreams;  // launch tables: two batches in flight per stream
    bool ok = hipMalloc(&S->pool, S->budget) == hipSuccess;
    if (!ok) S->pool = nullptr;
    ok = ok && hipMalloc(&S->d_tables, (size_t)slots * max_batch * sizeof(HcLayer)) == hipSuccess;
    ok = ok && hipHostMalloc(&S->h_tables, (size_t)slots * max_batch * sizeof(HcLayer), hipHostMallocDefault) ==
                   hipSuccess;
    for (int i = 0; ok && i < nstreams; ++i) {
        hipStream_t s;
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
        if (ok) S->streams.push_back(s);
    }
    for (int i = 0; ok && i < slots; ++i) S->free_slots.push_back(slots - 1 - i);
    for (int i = 0; ok && i < slots * max_batch; ++i) {  // one completion event per request in flight
        hipEvent_t e;
        ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) S->event_pool.push_back(e);
    }
    (void)hipSetDevice(prev);
    if (!ok) {
        destroy(S);
        return ENSEI_ERR_HIP;
    }
    S->book.reset(S->budget);
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return ENSEI_OK;
}

int ensei_server_create(ensei_ctx *ctx, size_t budget_bytes, int nstreams, int max_batch, ensei_server **out) {
    return server_create(ctx, budget_bytes, nstreams, max_batch, out, false);
}

int ensei_server_create_seeded(ensei_ctx *ctx, size_t budget_bytes, int nstreams, int max_batch,
                               ensei_server **out) {
    return server_create(ctx, budget_bytes, nstreams, max_batch, out, true);
}

int ensei_server_add_shape(ensei_server *S, const ensei_shape *shape, const int32_t *w, int *shape_id) {
    if (!S || !shape || !w || !shape_id) return ENSEI_ERR_ARG;
    const ensei_shape &d = *shape;
    if (d.H <= 0 || d.W <= 0 || d.Cin <= 0 || d.Cout <= 0 || d.n <= 0 || d.kh <= 0 || d.kw <= 0) return ENSEI_ERR_ARG;
    if (homconv_sizes(1, d.Cin, d.Cout, (int64_t)d.H * d.W, d.n)) return homconv_sizes(1, d.Cin, d.Cout, (int64_t)d.H * d.W, d.n);
    Shape sh;
    sh.d = d;
    sh.F = (int64_t)d.H * d.W;
    sh.footprint = parts_of(d, S->seeded).total;
    if (sh.footprint > S->book.budget()) return ENSEI_ERR_BUDGET;
    sh.narrow = d.Cin <= kNarrowCin;
    sh.wpack_bytes = wpack_bytes_as(d.Cout, d.Cin, sh.F, !sh.narrow);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->ctx->device);
    int rc = ENSEI_OK;
    // w is read on a private stream: pending work of every stream that may
    // still write it finishes first
    if (hipDeviceSynchronize() != hipSuccess) rc = ENSEI_ERR_HIP;
    if (!rc && hipMalloc(&sh.w_hat, (size_t)d.Cout * d.Cin * sh.F * 4) != hipSuccess) sh.w_hat = nullptr;
    if (!rc && sh.w_hat && hipMalloc(&sh.w_pack, sh.wpack_bytes) != hipSuccess) sh.w_pack = nullptr;
    if (!rc && (!sh.w_hat || !sh.w_pack)) rc = ENSEI_ERR_HIP;
    hipStream_t st = nullptr;
    if (!rc && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        st = nullptr;
        rc = ENSEI_ERR_HIP;
    }
    if (!rc) rc = ensei_weight_prep(S->ctx, w, d.Cout, d.Cin, d.kh, d.kw, d.H, d.W, sh.w_hat, st);
    if (!rc) rc = pack_weights_as(S->ctx, sh.w_hat, d.Cout, d.Cin, sh.F, !sh.narrow, sh.w_pack, st);
    if (st) {
        if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = ENSEI_ERR_HIP;
        (void)hipStreamDestroy(st);
    }
    (void)hipSetDevice(prev);
    if (rc) {
        if (sh.w_hat) (void)hipFree(sh.w_hat);
        if (sh.w_pack) (void)hipFree(sh.w_pack);
        return rc;
    }
    std::lock_guard<std::mutex> g(S->mu);
    S->shapes.push_back(sh);
    *shape_id = (int)S->shapes.size() - 1;
    return ENSEI_OK;
}

int ensei_server_submit(ensei_server *S, int shape_id, const ensei_request *req, uint64_t *ticket) {
    if (!S || !req || !ticket) return ENSEI_ERR_ARG;
    if (!req->x || !req->s || !req->e || !req->r || !req->s_a || !req->s_b) return ENSEI_ERR_ARG;
    const double t_arrival = now_s(S);  // before waiting for the lock
    std::lock_guard<std::mutex> g(S->mu);
    if (shape_id < 0 || shape_id >= (int)S->shapes.size()) return ENSEI_ERR_ARG;
    if (S->stop) return ENSEI_ERR_ARG;
    const uint64_t t = S->next_ticket;
    const int rc = S->book.submit(t, shape_id, S->shapes[shape_id].footprint, t_arrival);
    if (rc == ENSEI_ERR_BUDGET) ++S->n_refused;
    if (rc) return rc;
    Pending p;
    p.io = *req;
    {
        // the request's kernels wait for the caller's pending input work
        if (S->ready_pool.empty()) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                S->book.cancel(t, t_arrival);
                S->book.forget(t);
                return ENSEI_ERR_HIP;
            }
            S->ready_pool.push_back(e);
        }
        p.ready = S->ready_pool.back();
        if (hipEventRecord(p.ready, static_cast<hipStream_t>(req->stream)) != hipSuccess) {
            S->book.cancel(t, t_arrival);
            S->book.forget(t);
            return ENSEI_ERR_HIP;
        }
        S->ready_pool.pop_back();
    }
    S->pending.emplace(t, p);
    ++S->next_ticket;
    *ticket = t;
    S->cv_work.notify_one();
    return ENSEI_OK;
}

int ensei_server_cancel(ensei_server *S, uint64_t ticket) {
    if (!S) return ENSEI_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    const sched::Ticket *k = S->book.find(ticket);
    if (!k) return ENSEI_ERR_ARG;
    const bool queued = k->state == sched::kQueued;
    const int rc = S->book.cancel(ticket, now_s(S));
    if (rc) return rc;
    ++S->n_cancelled;
    if (queued) {
        // it never runs: its input event goes back, and requests that waited
        // behind it may be admitted now
        auto pit = S->pending.find(ticket);
        if (pit != S->pending.end()) {
            if (pit->second.ready) S->ready_pool.push_back(pit->second.ready);
            S->pending.erase(pit);
        }
        S->cv_done.notify_all();
        S->cv_work.notify_one();
    }
    return ENSEI_OK;
}

int ensei_server_set_queue_limit(ensei_server *S, size_t bytes) {
    if (!S) return ENSEI_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    S->book.set_queue_limit(bytes);
    return ENSEI_OK;
}

int ensei_server_clock(ensei_server *S, double *now) {
    if (!S || !now) return ENSEI_ERR_ARG;
    *now = now_s(S);
    return ENSEI_OK;
}

int ensei_server_poll(ensei_server *S, uint64_t ticket, ensei_request_info *info) {
    if (!S || !info) return ENSEI_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    const sched::Ticket *k = S->book.find(ticket);
    if (!k) return ENSEI_ERR_ARG;
    info->state = k->state;
    info->status = k->status;
    info->t_submit = k->t_submit;
    info->t_start = k->state == sched::kRunning || k->t_start > 0 ? k->t_start : 0.0;
    info->t_done = k->state >= sched::kDone ? k->t_done : 0.0;
    return ENSEI_OK;
}

int ensei_server_wait(ensei_server *S, uint64_t ticket, int timeout_ms) {
    if (!S) return ENSEI_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto done = [&] {
        const sched::Ticket *k = S->book.find(ticket);
        return !k || k->state >= sched::kDone;
    };
    if (!S->book.find(ticket)) return ENSEI_ERR_ARG;
    if (timeout_ms < 0)
        S->cv_done.wait(lk, done);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
        return ENSEI_ERR_TIMEOUT;
    const sched::Ticket *k = S->book.find(ticket);
    return k ? k->status : ENSEI_ERR_ARG;
}

int ensei_server_forget(ensei_server *S, uint64_t ticket) {
    if (!S) return ENSEI_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    return S->book.forget(ticket);
}

int ensei_server_stats(ensei_server *S, ensei_server_info *out) {
    if (!S || !out) return ENSEI_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    out->budget_bytes = S->budget;
    out->used_bytes = S->book.used();
    out->peak_used_bytes = S->book.peak_used();
    out->queued = S->book.queued();
    out->inflight_batches = S->inflight.size();
    out->completed = S->n_done;
    out->failed = S->n_failed;
    out->batches = S->n_batches;
    out->cancelled = S->n_cancelled;
    out->refused = S->n_refused;
    return ENSEI_OK;
}

int ensei_server_destroy(ensei_server *S) {
    if (!S) return ENSEI_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->ctx->device);
    destroy(S);
    (void)hipSetDevice(prev);
    return ENSEI_OK;
}

}  // extern "C"
