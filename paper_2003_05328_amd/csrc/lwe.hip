// LWE encryption and decryption over q = 2^64 (one ciphertext per frequency
// coefficient): streaming, HBM-bound matrix-vector kernels.
//
// One wave owns one ciphertext row of n+1 words at a time: lane l touches
// words l, l+64, ... so every wave instruction moves 512 contiguous bytes.
// The key s (n ternary bytes) sits in LDS; the row's inner product <a, s>
// is accumulated per lane and summed across the wave with DPP/ds_swizzle
// shuffles. Encryption generates the uniform a-words on the fly with a
// counter-based SplitMix64, so its only HBM traffic is the ciphertext
// written (plus 8 bytes of m and e per row).
#include "ensei_internal.hpp"

namespace ensei {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014): output number k
// of the generator seeded with x is mix(x + k * gamma).
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// s_j * a mod 2^64 for s_j in {-1, 0, 1}.
__device__ __forceinline__ uint64_t ternary_times(int8_t sj, uint64_t a) {
    const uint64_t nz = sj != 0 ? ~0ull : 0ull;
    const uint64_t neg = sj < 0 ? ~0ull : 0ull;
    return ((a & nz) ^ neg) - neg;  // (x ^ -1) + 1 = -x
}

constexpr int kWavesPerBlock = 4;

__global__ __launch_bounds__(256) void encrypt_kernel(const uint32_t *__restrict__ m, const int8_t *__restrict__ s,
                                                      const int32_t *__restrict__ e, int64_t num_ct, int n,
                                                      uint64_t seed_a, uint64_t ct_index0, uint64_t delta,
                                                      uint64_t *__restrict__ ct) {
    extern __shared__ int8_t key[];
    for (int i = threadIdx.x; i < n; i += blockDim.x) key[i] = s[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const uint64_t step = kGamma * 64;
    const int64_t rowlen = (int64_t)n + 1;
    for (int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); c < num_ct; c += stride) {
        uint64_t *row = ct + c * rowlen;
        uint64_t z = seed_a + ((ct_index0 + (uint64_t)c) * (uint64_t)n + (uint64_t)lane + 1) * kGamma;
        uint64_t acc = 0;
#pragma unroll 4
        for (int j = lane; j < n; j += 64) {
            const uint64_t a = splitmix_mix(z);
            row[j] = a;
            acc += ternary_times(key[j], a);
            z += step;
        }
        acc = wave_sum_u64(acc);
        if (lane == 0) row[n] = acc + (uint64_t)(int64_t)e[c] + delta * (uint64_t)m[c];
    }
}

// Round half up of phi * p / 2^64, then mod p (p < 2^31):
// with X = phi_lo * p and Y = phi_hi * p, phi * p + 2^63 = (Y + (X >> 32) + 2^31) 2^32 + (X mod 2^32),
// so the quotient by 2^64 is (Y + (X >> 32) + 2^31) >> 32, which is at most p.
__device__ __forceinline__ uint32_t decode(uint64_t phi, uint32_t p) {
    const uint64_t X = (uint64_t)(uint32_t)phi * p;
    const uint64_t Y = (phi >> 32) * p;
    const uint32_t v = (uint32_t)((Y + (X >> 32) + 0x80000000ull) >> 32);
    return v >= p ? v - p : v;
}

__global__ __launch_bounds__(256) void decrypt_kernel(const uint64_t *__restrict__ ct, const int8_t *__restrict__ s,
                                                      int64_t num_ct, int n, uint32_t p, uint32_t *__restrict__ m) {
    extern __shared__ int8_t key[];
    for (int i = threadIdx.x; i < n; i += blockDim.x) key[i] = s[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t rowlen = (int64_t)n + 1;
    for (int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); c < num_ct; c += stride) {
        const uint64_t *row = ct + c * rowlen;
        const uint64_t bword = row[n];  // same address in every lane: one transaction, issued first
        uint64_t acc = 0;
        int j = lane;
        // 16 words per lane in flight at once
        for (; j + 64 * 15 < n; j += 64 * 16) {
            uint64_t w[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) w[k] = row[j + 64 * k];
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += ternary_times(key[j + 64 * k], w[k]);
        }
        for (; j < n; j += 64) acc += ternary_times(key[j], row[j]);
        acc = wave_sum_u64(acc);
        if (lane == 0) m[c] = decode(bword - acc, p);
    }
}

static int64_t lwe_grid(int64_t num_ct) {
    int64_t blocks = (num_ct + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t cap = 256 * 16;  // CUs x resident blocks: enough waves to keep HBM busy
    return blocks < cap ? blocks : cap;
}

}  // namespace ensei

using namespace ensei;

extern "C" {

int ensei_encrypt(ensei_ctx *ctx, const uint32_t *m, const int8_t *s, const int32_t *e, int64_t num_ct, int n,
                  uint64_t seed_a, uint64_t ct_index0, uint64_t *ct, void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!m || !s || !e || !ct || num_ct <= 0 || n <= 0) return ENSEI_ERR_ARG;
    if (n > ENSEI_MAX_LWE_N) return ENSEI_ERR_LIMIT;
    if (((uintptr_t)m & 3) || ((uintptr_t)e & 3) || ((uintptr_t)ct & 7)) return ENSEI_ERR_ALIGN;
    const size_t ctb = (size_t)num_ct * (n + 1) * 8;
    if (overlaps(ct, ctb, m, (size_t)num_ct * 4) || overlaps(ct, ctb, e, (size_t)num_ct * 4) ||
        overlaps(ct, ctb, s, (size_t)n))
        return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(encrypt_kernel, dim3((unsigned)lwe_grid(num_ct)), dim3(256), (size_t)n, (hipStream_t)stream, m,
                       s, e, num_ct, n, seed_a, ct_index0, ctx->delta, ct);
    return launch_status();
}

int ensei_decrypt(ensei_ctx *ctx, const uint64_t *ct, const int8_t *s, int64_t num_ct, int n, uint32_t *m,
                  void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!m || !s || !ct || num_ct <= 0 || n <= 0) return ENSEI_ERR_ARG;
    if (n > ENSEI_MAX_LWE_N) return ENSEI_ERR_LIMIT;
    if (((uintptr_t)m & 3) || ((uintptr_t)ct & 7)) return ENSEI_ERR_ALIGN;
    const size_t ctb = (size_t)num_ct * (n + 1) * 8;
    if (overlaps(m, (size_t)num_ct * 4, ct, ctb) || overlaps(m, (size_t)num_ct * 4, s, (size_t)n))
        return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(decrypt_kernel, dim3((unsigned)lwe_grid(num_ct)), dim3(256), (size_t)n, (hipStream_t)stream, ct,
                       s, num_ct, n, ctx->p, m);
    return launch_status();
}

}  // extern "C"
