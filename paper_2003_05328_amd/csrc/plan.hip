// Batched plans: a stack of independent secure convolutions captured as one
// HIP graph, with the HomConv of all layers in one persistent launch and its
// tile schedule picked by timing candidates on the plan's own shapes.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "ensei_internal.hpp"

struct ensei_plan {
    ensei_ctx *ctx = nullptr;
    std::vector<ensei_layer> layers;
    std::vector<uint32_t *> w_hat;
    std::vector<int8_t *> w_pack;
    std::vector<ensei::HcLayer> problems;  // in the one persistent launch
    // narrow-input and deep layers, each launched on its own kernel (with
    // paired fragments or not)
    std::vector<std::pair<ensei::HcLayer, bool>> single;
    ensei::HcLayer *d_table = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the same work as three graphs, one per stage (ensei_plan_run_stage)
    hipGraph_t stage_graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t stage_exec[3] = {nullptr, nullptr, nullptr};
    // concurrent branches: within each stage the layers (and in the HomConv
    // stage the shared launch and each layer of its own) are independent, so
    // they fork onto side streams and join back; kept when faster
    bool concurrent = false;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> joins;  // [0] fork, [1 + i] side stream i's join
    ensei::HcSchedule sched{0, 0};
    ensei_schedule info{};
    // seeded ciphertexts: each layer's ct_in holds only the b words,
    // [batch][F][Cin], and HomConv regenerates the a-words from seed_a
    bool seeded = false;
};

namespace ensei {
namespace {

constexpr int kSideStreams = 3;  // with the plan's own stream, the device's four hardware queues

struct DeviceGuard {
    int prev = 0;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() { (void)hipSetDevice(prev); }
};

void release(ensei_plan *P) {
    if (P->stream) (void)hipStreamSynchronize(P->stream);  // setup work may still read the buffers
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (int k = 0; k < 3; ++k) {
        if (P->stage_exec[k]) (void)hipGraphExecDestroy(P->stage_exec[k]);
        if (P->stage_graph[k]) (void)hipGraphDestroy(P->stage_graph[k]);
    }
    for (hipStream_t q : P->side) {
        (void)hipStreamSynchronize(q);
        (void)hipStreamDestroy(q);
    }
    for (hipEvent_t e : P->joins) (void)hipEventDestroy(e);
    for (auto *q : P->w_hat) (void)hipFree(q);
    for (auto *q : P->w_pack) (void)hipFree(q);
    if (P->d_table) (void)hipFree(P->d_table);
    if (P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
}

// Runs nb independent branches fn(i, stream): in order on st, or, with the
// plan's concurrent branches, dealt round-robin over its side streams, which
// first wait for the work already queued on st and are joined back into st
// at the end (during graph capture this forks and joins the graph).
template <class Fn>
int fork_join(ensei_plan *P, hipStream_t st, int nb, Fn fn) {
    const int ns = P->concurrent ? (int)std::min<size_t>(P->side.size(), (size_t)nb) : 0;
    if (ns < 2) {
        for (int i = 0; i < nb; ++i) {
            const int rc = fn(i, st);
            if (rc) return rc;
        }
        return ENSEI_OK;
    }
    if (hipEventRecord(P->joins[0], st) != hipSuccess) return ENSEI_ERR_HIP;
    for (int j = 0; j < ns; ++j)
        if (hipStreamWaitEvent(P->side[j], P->joins[0], 0) != hipSuccess) return ENSEI_ERR_HIP;
    int rc = ENSEI_OK;
    for (int i = 0; i < nb && !rc; ++i) rc = fn(i, P->side[i % ns]);
    for (int j = 0; j < ns; ++j) {  // always join, so that a capture can end
        if (hipEventRecord(P->joins[1 + j], P->side[j]) != hipSuccess ||
            hipStreamWaitEvent(st, P->joins[1 + j], 0) != hipSuccess)
            rc = rc ? rc : ENSEI_ERR_HIP;
    }
    return rc;
}

// Client side of every layer: x^ = NTT2D(x), ct_in = Enc(x^).
int run_front(ensei_plan *P, hipStream_t st) {
    return fork_join(P, st, (int)P->layers.size(), [P](int i, hipStream_t q) {
        const ensei_layer &l = P->layers[i];
        const int64_t F = (int64_t)l.H * l.W;
        int rc = ensei_ntt2d(P->ctx, l.x, l.x_hat, l.batch * l.Cin, l.H, l.W, q);
        if (!rc)
            rc = P->seeded
                     ? ensei_encrypt_seeded(P->ctx, l.x_hat, l.s, l.e, l.batch, l.Cin, F, l.n, l.seed_a, 0, l.ct_in, q)
                     : ensei_encrypt(P->ctx, l.x_hat, l.s, l.e, l.batch, l.Cin, F, l.n, l.seed_a, 0, l.ct_in, q);
        return rc;
    });
}

// Dec, the client's INTT2D and the server's share of every layer.
int run_back(ensei_plan *P, hipStream_t st) {
    return fork_join(P, st, (int)P->layers.size(), [P](int i, hipStream_t q) {
        const ensei_layer &l = P->layers[i];
        const int64_t F = (int64_t)l.H * l.W;
        int rc = ensei_decrypt(P->ctx, l.ct_out, l.s, l.batch, l.Cout, F, l.n, l.m, q);
        if (!rc) rc = ensei_intt2d(P->ctx, l.m, l.s_a, l.batch * l.Cout, l.H, l.W, q);
        if (!rc) rc = ensei_server_share(P->ctx, l.r, l.s_b, l.batch * l.Cout, l.H, l.W, q);
        return rc;
    });
}

// The HomConv stage: branch 0 the shared launch (s.chunk = -1: the shared
// problems each in a launch of their own instead), then each layer on a
// kernel of its own.
int run_homconv(ensei_plan *P, HcSchedule s, hipStream_t st) {
    const int nb = 1 + (int)P->single.size();
    return fork_join(P, st, nb, [P, s](int i, hipStream_t q) {
        int rc = ENSEI_OK;
        if (i == 0) {
            if (s.chunk < 0) {
                for (HcLayer h : P->problems) {
                    h.tile0 = 0;  // its own tile space
                    if (!rc) rc = homconv_launch(P->ctx, &h, nullptr, 1, true, HcSchedule{0, 0}, q, P->seeded);
                }
            } else if (!P->problems.empty()) {
                rc = homconv_launch(P->ctx, P->problems.data(), P->d_table, (int)P->problems.size(), true, s, q,
                                    P->seeded);
            }
            return rc;
        }
        const auto &hp = P->single[i - 1];
        return homconv_launch(P->ctx, &hp.first, nullptr, 1, hp.second, HcSchedule{0, 0}, q, P->seeded);
    });
}

// Cache key: device, modulus and the HomConv shape of every layer in the
// shared persistent launch.
std::string plan_key(const ensei_plan *P) {
    hipDeviceProp_t prop;
    char buf[160];
    const char *arch = hipGetDeviceProperties(&prop, P->ctx->device) == hipSuccess ? prop.gcnArchName : "unknown";
    snprintf(buf, sizeof buf, "%s/cus=%d/p=%u%s", arch, P->ctx->num_cus, P->ctx->p, P->seeded ? "/seeded" : "");
    std::string key = buf;
    for (const HcLayer &h : P->problems) {
        snprintf(buf, sizeof buf, "|b%lld.f%lld.i%d.o%d.n%d", (long long)h.B, (long long)h.F, h.Cin, h.Cout, h.n);
        key += buf;
    }
    for (char &c : key)
        if (c == ' ') c = '_';
    return key;
}

// A cache line is "key blocks chunk [us [branches]]"; branches (0 or 1), when
// present, pins the serial or concurrent capture too (else it is timed).
bool cache_lookup(const char *path, const std::string &key, HcSchedule *s, int *branches) {
    FILE *fh = fopen(path, "r");
    if (!fh) return false;
    char line[4096];
    bool found = false;
    while (fgets(line, sizeof line, fh)) {
        char k[3900];
        int blocks, br = -1;
        long long chunk;
        double us;
        const int got = sscanf(line, "%3899s %d %lld %lf %d", k, &blocks, &chunk, &us, &br);
        if (got >= 3 && (key == k || strcmp(k, "*") == 0) && blocks > 0 && chunk >= -1) {
            *s = HcSchedule{blocks, (int64_t)chunk};
            *branches = got == 5 && (br == 0 || br == 1) ? br : -1;
            found = true;  // the last entry for a key wins
        }
    }
    fclose(fh);
    return found;
}

void cache_append(const char *path, const std::string &key, HcSchedule s, double us) {
    FILE *fh = fopen(path, "a");
    if (!fh) return;
    fprintf(fh, "%s %d %lld %.1f\n", key.c_str(), s.blocks, (long long)s.chunk, us);
    fclose(fh);
}

// Mean time of the HomConv launch under schedule s (one warm-up, three timed).
int time_schedule(ensei_plan *P, HcSchedule s, double *us) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return ENSEI_ERR_HIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return ENSEI_ERR_HIP;
    }
    int rc = run_homconv(P, s, P->stream);
    const int reps = 3;
    if (!rc && hipEventRecord(a, P->stream) != hipSuccess) rc = ENSEI_ERR_HIP;
    for (int i = 0; i < reps && !rc; ++i) rc = run_homconv(P, s, P->stream);
    if (!rc && hipEventRecord(b, P->stream) != hipSuccess) rc = ENSEI_ERR_HIP;
    float ms = 0;
    if (!rc && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
        rc = ENSEI_ERR_HIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *us = ms * 1e3 / reps;
    return rc;
}

// Mean time of one replay of a captured plan (one warm-up, three timed).
int time_graph(ensei_plan *P, hipGraphExec_t exec, double *us) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return ENSEI_ERR_HIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return ENSEI_ERR_HIP;
    }
    int rc = hipGraphLaunch(exec, P->stream) == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP;
    const int reps = 3;
    if (!rc && hipEventRecord(a, P->stream) != hipSuccess) rc = ENSEI_ERR_HIP;
    for (int i = 0; i < reps && !rc; ++i)
        if (hipGraphLaunch(exec, P->stream) != hipSuccess) rc = ENSEI_ERR_HIP;
    if (!rc && hipEventRecord(b, P->stream) != hipSuccess) rc = ENSEI_ERR_HIP;
    float ms = 0;
    if (!rc && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
        rc = ENSEI_ERR_HIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *us = ms * 1e3 / reps;
    return rc;
}

// Captures stage k of the plan (0 client front, 1 HomConv, 2 back; -1 all
// three in order) as a graph and instantiates it.
int capture(ensei_plan *P, int k, hipGraph_t *graph, hipGraphExec_t *exec) {
    if (hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return ENSEI_ERR_HIP;
    int rc = ENSEI_OK;
    if (k < 0 || k == 0) rc = run_front(P, P->stream);
    if (!rc && (k < 0 || k == 1)) rc = run_homconv(P, P->sched, P->stream);
    if (!rc && (k < 0 || k == 2)) rc = run_back(P, P->stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(P->stream, &g);
    *graph = g;
    if (!rc && (ec != hipSuccess || !g)) rc = ENSEI_ERR_HIP;
    if (!rc && hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
        *exec = nullptr;
        rc = ENSEI_ERR_HIP;
    }
    return rc;
}

// Creates a plan (ensei_plan_create, ensei_plan_create_seeded).
int plan_create(ensei_ctx *ctx, const ensei_layer *layers, int nlayers, const char *tune_cache, ensei_plan **out,
                bool seeded) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out || !layers || nlayers < 1) return ENSEI_ERR_ARG;
    if (nlayers > ENSEI_MAX_PLAN_LAYERS) return ENSEI_ERR_LIMIT;
    *out = nullptr;
    DeviceGuard guard(ctx->device);
    // the layers' buffers are read on the plan's own stream: let pending work
    // of every stream (the caller's included) finish first
    if (hipDeviceSynchronize() != hipSuccess) return ENSEI_ERR_HIP;
    ensei_plan *P = new ensei_plan;
    P->ctx = ctx;
    P->seeded = seeded;
    P->layers.assign(layers, layers + nlayers);
    if (hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) != hipSuccess) {
        P->stream = nullptr;
        release(P);
        return ENSEI_ERR_HIP;
    }
    for (int i = 0; i < kSideStreams; ++i) {  // default priority, like every stream here
        hipStream_t q;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
            release(P);
            return ENSEI_ERR_HIP;
        }
        P->side.push_back(q);
    }
    for (int i = 0; i <= kSideStreams; ++i) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            release(P);
            return ENSEI_ERR_HIP;
        }
        P->joins.push_back(e);
    }
    // server setup: transformed and packed filters (paired layout, folded for
    // narrow inputs); narrow and deep layers run on their own kernels, the
    // others share one persistent launch
    int64_t tile0 = 0;
    for (const ensei_layer &l : P->layers) {
        if (l.H <= 0 || l.W <= 0 || l.Cin <= 0 || l.Cout <= 0 || l.batch <= 0) {
            release(P);
            return ENSEI_ERR_ARG;
        }
        const int64_t F = (int64_t)l.H * l.W;
        const bool narrow = l.Cin <= kNarrowCin;
        uint32_t *wh = nullptr;
        int8_t *wp = nullptr;
        const size_t wpb = wpack_bytes_as(l.Cout, l.Cin, F, !narrow);
        if (hipMalloc(&wh, (size_t)l.Cout * l.Cin * F * 4) != hipSuccess) wh = nullptr;
        if (wh && hipMalloc(&wp, wpb) != hipSuccess) wp = nullptr;
        if (wh) P->w_hat.push_back(wh);
        if (wp) P->w_pack.push_back(wp);
        if (!wh || !wp) {
            release(P);
            return ENSEI_ERR_HIP;
        }
        rc = ensei_weight_prep(ctx, l.w, l.Cout, l.Cin, l.kh, l.kw, l.H, l.W, wh, P->stream);
        if (!rc) rc = pack_weights_as(ctx, wh, l.Cout, l.Cin, F, !narrow, wp, P->stream);
        HcLayer h;
        if (!rc) rc = homconv_problem(ctx, &h, l.ct_in, wp, l.r, l.batch, l.Cin, l.Cout, F, l.n, l.ct_out, wpb, seeded);
        h.seed_a = seeded ? l.seed_a : 0;
        h.idx0 = 0;
        if (rc) {
            release(P);
            return rc;
        }
        if (narrow || homconv_deep_fits(h, seeded)) {
            P->single.emplace_back(h, !narrow);
            continue;
        }
        h.n_items = frag_items(l.Cin, true);
        h.tile0 = tile0;
        tile0 += h.n_tiles;
        P->problems.push_back(h);
    }
    const size_t tb = P->problems.size() * sizeof(HcLayer);
    if (tb && hipMalloc(&P->d_table, tb) != hipSuccess) {
        P->d_table = nullptr;
        release(P);
        return ENSEI_ERR_HIP;
    }
    if ((tb && hipMemcpyAsync(P->d_table, P->problems.data(), tb, hipMemcpyHostToDevice, P->stream) != hipSuccess) ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
        release(P);
        return ENSEI_ERR_HIP;
    }

    // one eager pass: every argument check of the single calls, on real buffers
    rc = run_front(P, P->stream);
    if (!rc) rc = run_homconv(P, HcSchedule{0, 0}, P->stream);
    if (!rc) rc = run_back(P, P->stream);
    if (!rc && hipStreamSynchronize(P->stream) != hipSuccess) rc = ENSEI_ERR_HIP;
    if (rc) {
        release(P);
        return rc;
    }

    // the HomConv tile schedule: cached, or the fastest candidate
    const std::string key = plan_key(P);
    int pin_branches = -1;
    HcSchedule best{ctx->num_cus, 0};
    double best_us = 0;
    if (P->problems.empty()) {
        // nothing to schedule: every layer runs on its own kernel
        rc = time_schedule(P, best, &best_us);
        if (rc) {
            release(P);
            return rc;
        }
    } else if (tune_cache && cache_lookup(tune_cache, key, &best, &pin_branches)) {
        P->info.from_cache = 1;
    } else {
        // chunk -1: no shared launch, each problem on its own
        const int64_t chunks[] = {0, 1, 4, 16, 64, 256, -1};
        bool first = true;
        for (int64_t c : chunks) {
            const HcSchedule s{ctx->num_cus, c};
            double us = 0;
            rc = time_schedule(P, s, &us);
            if (rc) {
                release(P);
                return rc;
            }
            if (first || us < best_us) {
                best = s;
                best_us = us;
                first = false;
            }
        }
        if (tune_cache) cache_append(tune_cache, key, best, best_us);
    }
    P->sched = best;
    P->info.blocks = best.blocks;
    P->info.chunk = best.chunk;
    P->info.homconv_us = best_us;
    P->info.shared_layers = (int)P->problems.size();
    P->info.own_layers = (int)P->single.size();

    // capture the whole stack as one graph, with the layers of each stage in
    // order or as concurrent branches: pinned by the cache, else whichever
    // replays faster; then each stage as a graph of its own in the same form
    rc = capture(P, -1, &P->graph, &P->exec);
    if (!rc && pin_branches >= 0) {
        P->concurrent = pin_branches == 1;
        if (P->concurrent) {
            (void)hipGraphExecDestroy(P->exec);
            (void)hipGraphDestroy(P->graph);
            P->exec = nullptr;
            P->graph = nullptr;
            rc = capture(P, -1, &P->graph, &P->exec);
        }
    } else if (!rc && P->layers.size() > 1) {
        double serial_us = 0, conc_us = 0;
        hipGraph_t g2 = nullptr;
        hipGraphExec_t e2 = nullptr;
        rc = time_graph(P, P->exec, &serial_us);
        P->concurrent = true;
        if (!rc) rc = capture(P, -1, &g2, &e2);
        if (!rc) rc = time_graph(P, e2, &conc_us);
        if (!rc && conc_us < serial_us) {
            std::swap(g2, P->graph);
            std::swap(e2, P->exec);
        } else {
            P->concurrent = false;
        }
        if (e2) (void)hipGraphExecDestroy(e2);
        if (g2) (void)hipGraphDestroy(g2);
        P->info.serial_us = serial_us;
        P->info.branches_us = conc_us;
    }
    P->info.branches = P->concurrent ? 1 : 0;
    for (int k = 0; k < 3 && !rc; ++k) rc = capture(P, k, &P->stage_graph[k], &P->stage_exec[k]);
    if (rc) {
        release(P);
        return rc;
    }
    *out = P;
    return ENSEI_OK;
}
}  // namespace
}  // namespace ensei

using namespace ensei;

extern "C" {

int ensei_plan_create(ensei_ctx *ctx, const ensei_layer *layers, int nlayers, const char *tune_cache,
                      ensei_plan **out) {
    return plan_create(ctx, layers, nlayers, tune_cache, out, false);
}

int ensei_plan_create_seeded(ensei_ctx *ctx, const ensei_layer *layers, int nlayers, const char *tune_cache,
                             ensei_plan **out) {
    return plan_create(ctx, layers, nlayers, tune_cache, out, true);
}

int ensei_plan_run(ensei_plan *plan, void *stream) {
    if (!plan || !plan->exec) return ENSEI_ERR_ARG;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP;
}

int ensei_plan_run_stage(ensei_plan *plan, int stage, void *stream) {
    if (!plan || stage < 0 || stage > 2 || !plan->stage_exec[stage]) return ENSEI_ERR_ARG;
    return hipGraphLaunch(plan->stage_exec[stage], (hipStream_t)stream) == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP;
}

int ensei_plan_schedule(const ensei_plan *plan, ensei_schedule *out) {
    if (!plan || !out) return ENSEI_ERR_ARG;
    *out = plan->info;
    return ENSEI_OK;
}

int ensei_plan_destroy(ensei_plan *plan) {
    if (!plan) return ENSEI_OK;
    DeviceGuard guard(plan->ctx->device);
    release(plan);
    return ENSEI_OK;
}

}  // extern "C"
