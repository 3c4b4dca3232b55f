// Context, status codes and shared host-side checks of libensei.
#include <stdlib.h>
#include <string.h>

#include <math.h>

#include "ensei_internal.hpp"

namespace ensei {

static uint64_t host_mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((unsigned __int128)a * b % p); }

static uint64_t host_powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    for (; e; e >>= 1) {
        if (e & 1) r = host_mulmod(r, a, p);
        a = host_mulmod(a, a, p);
    }
    return r;
}

static bool host_is_prime(uint64_t p) {
    if (p < 2) return false;
    for (uint64_t d = 2; d * d <= p; ++d)
        if (p % d == 0) return false;
    return true;
}

// Smallest g whose order is p - 1: g^((p-1)/q) != 1 for every prime q | p-1.
static uint32_t host_generator(uint32_t p) {
    uint32_t m = p - 1, primes[32];
    int np = 0;
    for (uint32_t d = 2; d * d <= m; ++d)
        if (m % d == 0) {
            primes[np++] = d;
            while (m % d == 0) m /= d;
        }
    if (m > 1) primes[np++] = m;
    for (uint32_t g = 2; g < p; ++g) {
        bool ok = true;
        for (int i = 0; i < np && ok; ++i) ok = host_powmod(g, (p - 1) / primes[i], p) != 1;
        if (ok) return g;
    }
    return 0;
}

int check_ctx(const ensei_ctx *ctx) {
    if (!ctx) return ENSEI_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ENSEI_ERR_HIP;
    return dev == ctx->device ? ENSEI_OK : ENSEI_ERR_DEVICE;
}

bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

int launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP;
}

int ilog2_pow2(int v) {
    if (v < 2 || (v & (v - 1))) return -1;
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace ensei

using namespace ensei;

extern "C" {

const char *ensei_status_str(int s) {
    switch (s) {
        case ENSEI_OK: return "ok";
        case ENSEI_ERR_ARG: return "invalid argument (null pointer, non-positive size or bad flag)";
        case ENSEI_ERR_SHAPE: return "unsupported transform shape (H, W must be powers of two in [2,128] dividing p-1)";
        case ENSEI_ERR_MODULUS: return "modulus must be a prime in [3, 2^22)";
        case ENSEI_ERR_ALIGN: return "misaligned pointer";
        case ENSEI_ERR_OVERLAP: return "output overlaps an input";
        case ENSEI_ERR_LIMIT: return "size beyond the supported range";
        case ENSEI_ERR_DEVICE: return "current HIP device is not the context's device";
        case ENSEI_ERR_HIP: return "HIP runtime error";
        case ENSEI_ERR_TIMEOUT: return "timed out before the request finished";
        case ENSEI_ERR_BUDGET: return "request does not fit the server's budget or queue limit";
        case ENSEI_ERR_CANCELLED: return "request was cancelled";
        case ENSEI_ERR_STATE: return "request has already finished";
        default: return "unknown status";
    }
}

int ensei_ctx_create(ensei_ctx **out, uint32_t p, int device) {
    if (!out) return ENSEI_ERR_ARG;
    *out = nullptr;
    if (p < 3 || p >= (1u << 22) || !host_is_prime(p)) return ENSEI_ERR_MODULUS;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return ENSEI_ERR_HIP;
    if (device < 0 || device >= ndev) return ENSEI_ERR_ARG;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return ENSEI_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return ENSEI_ERR_HIP;

    ensei_ctx *c = (ensei_ctx *)calloc(1, sizeof(ensei_ctx));
    if (!c) return ENSEI_ERR_HIP;
    c->device = device;
    c->p = p;
    c->g = host_generator(p);
    c->delta = (uint64_t)((((unsigned __int128)1) << 64) / p);
    int lg = 0;
    while (lg < 7 && (p - 1) % (1u << (lg + 1)) == 0) ++lg;
    c->max_log = lg;
    if (hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        c->num_cus <= 0)
        c->num_cus = 256;

    // Twiddles omega_L^j (and their 2^24-scaled quotients) per direction and length.
    uint2 tw[2 * kTwPerDir];
    memset(tw, 0, sizeof(tw));
    for (int d = 0; d < 2; ++d)
        for (int l = 1; l <= lg; ++l) {
            uint32_t L = 1u << l;
            uint64_t w = host_powmod(c->g, (p - 1) / L, p);
            if (d) w = host_powmod(w, p - 2, p);
            uint64_t x = 1;
            for (uint32_t j = 0; j < L / 2; ++j) {
                tw[d * kTwPerDir + (L / 2 - 1) + j] = make_uint2((uint32_t)x, (uint32_t)((x << 24) / p));
                x = host_mulmod(x, w, p);
            }
        }
    // Error sampler thresholds for the rounded Gaussian of sigma = 3.2:
    // P(|e| <= k) = erf((k + 1/2) / (sigma sqrt 2)) = erf(5 (2k + 1) / (32 sqrt 2)),
    // in long double (a 64-bit significand, far finer than the 2^-48 grid);
    // erf < 1 keeps every entry below 2^48.
    static_assert(sizeof(c->cdt) / sizeof(c->cdt[0]) == kCdtSize, "threshold count");
    for (int k = 0; k < kCdtSize; ++k) {
        const long double x = (long double)(5 * (2 * k + 1)) / (32.0L * sqrtl(2.0L));
        const long double v = floorl(ldexpl(erfl(x), kCdtBits));
        const uint64_t top = (1ull << kCdtBits) - 1;
        c->cdt[k] = v >= (long double)top ? top : (uint64_t)v;
    }
    int st = ENSEI_OK;
    if (hipMalloc(&c->d_tw, sizeof(tw)) != hipSuccess ||
        hipMemcpy(c->d_tw, tw, sizeof(tw), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&c->d_cdt, sizeof(c->cdt)) != hipSuccess ||
        hipMemcpy(c->d_cdt, c->cdt, sizeof(c->cdt), hipMemcpyHostToDevice) != hipSuccess)
        st = ENSEI_ERR_HIP;
    (void)hipSetDevice(prev);
    if (st != ENSEI_OK) {
        if (c->d_tw) (void)hipFree(c->d_tw);
        if (c->d_cdt) (void)hipFree(c->d_cdt);
        free(c);
        return st;
    }
    *out = c;
    return ENSEI_OK;
}

int ensei_ctx_destroy(ensei_ctx *ctx) {
    if (!ctx) return ENSEI_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipFree(ctx->d_tw);
    const hipError_t e2 = hipFree(ctx->d_cdt);
    if (e == hipSuccess) e = e2;
    (void)hipSetDevice(prev);
    free(ctx);
    return e == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP;
}

int ensei_error_table(const ensei_ctx *ctx, uint64_t *out, int n) {
    if (!ctx || !out || n < kCdtSize) return ENSEI_ERR_ARG;
    memcpy(out, ctx->cdt, sizeof(ctx->cdt));
    return kCdtSize;
}

int ensei_ctx_device(const ensei_ctx *ctx) { return ctx ? ctx->device : -1; }
uint32_t ensei_ctx_modulus(const ensei_ctx *ctx) { return ctx ? ctx->p : 0; }
uint64_t ensei_ctx_delta(const ensei_ctx *ctx) { return ctx ? ctx->delta : 0; }
int ensei_ctx_max_dim(const ensei_ctx *ctx) { return ctx ? (1 << ctx->max_log) : 0; }

}  // extern "C"
