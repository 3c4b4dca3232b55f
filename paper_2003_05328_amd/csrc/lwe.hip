// LWE encryption and decryption over q = 2^64 (one ciphertext per frequency
// coefficient): streaming, HBM-bound matrix-vector kernels over the
// word-major ciphertext layout ct[b][f][j][c].
//
// A workgroup owns a group of up to 64 ciphertexts that sit side by side in
// memory: 64 channels of one (b, f) when C >= 64, else floor(64 / C)
// consecutive frequencies of all C channels. Lane = ciphertext, so every
// wave instruction moves the group's word j of all its ciphertexts - one
// contiguous 512-byte run when C >= 64. The waves of the workgroup (4 for
// Enc, 16 for Dec) split the word range [0, n) into equal 4-aligned pieces;
// the key byte s_j is the same for every lane (read from
// LDS as a broadcast), each lane accumulates its own <a, s> and the waves'
// partial sums meet in LDS. Encryption generates the uniform a-words on the
// fly with a counter-based SplitMix64, so its only HBM traffic is the
// ciphertexts written (plus 8 bytes of m and e per ciphertext).
#include "ensei_internal.hpp"

namespace ensei {

// Group geometry shared by Enc and Dec.
struct LweGroups {
    int lanes_per_f;  // min(C, 64)
    int f_per_group;  // 64 / lanes_per_f (1 when C >= 64)
    int c_blocks;     // ceil(C / 64) (1 when C < 64)
    int64_t f_groups; // ceil(F / f_per_group)
};

__host__ __device__ inline LweGroups lwe_groups(int C, int64_t F) {
    LweGroups g;
    g.lanes_per_f = C < 64 ? C : 64;
    g.f_per_group = 64 / g.lanes_per_f;
    g.c_blocks = (C + 63) / 64;
    g.f_groups = (F + g.f_per_group - 1) / g.f_per_group;
    return g;
}

// Position of this lane's ciphertext: (b, f, c), and whether it exists.
struct LweLane {
    int64_t b, f;
    int c;
    bool ok;
};

__device__ __forceinline__ LweLane lwe_lane(const LweGroups &G, int C, int64_t F, int64_t group, int lane) {
    LweLane L;
    const int cb = (int)(group % G.c_blocks);
    const int64_t rest = group / G.c_blocks;
    const int64_t fg = rest % G.f_groups;
    L.b = rest / G.f_groups;
    const int fl = lane / G.lanes_per_f;
    L.c = cb * 64 + lane % G.lanes_per_f;
    L.f = fg * G.f_per_group + fl;
    L.ok = fl < G.f_per_group && L.f < F && L.c < C;
    return L;
}

constexpr int kWaves = 4;      // Enc: waves per workgroup
constexpr int kDecWaves = 16;  // Dec: more waves per group keep more loads in flight

// Key bytes s_j .. s_j+3 (the same for every lane) from the LDS copy of the
// key, moved to a scalar register; j is a multiple of 4.
__device__ __forceinline__ uint32_t key4(const int8_t *key, int j) {
    return __builtin_amdgcn_readfirstlane(*reinterpret_cast<const uint32_t *>(key + j));
}

// All-ones when the key byte k of `k4` is +1 (pos) / -1 (neg), else zero.
__device__ __forceinline__ uint64_t key_mask(uint32_t k4, int k, int sign) {
    const int sj = (int)(int8_t)(k4 >> (8 * k));
    return sj == sign ? ~0ull : 0ull;
}

// STORE_A = false (seeded ciphertexts): the a-words are only summed into
// <a, s>, not stored, and the b words go to ct as [B][F][C].
template <bool STORE_A>
__global__ __launch_bounds__(256) void encrypt_kernel(const uint32_t *__restrict__ m, const int8_t *__restrict__ s,
                                                      const int32_t *__restrict__ e, int C, int64_t F, int n,
                                                      uint64_t seed_a, uint64_t ct_index0, uint64_t delta,
                                                      uint64_t *__restrict__ ct, LweGroups G) {
    extern __shared__ uint8_t smem[];  // key bytes (n, padded to 8) then kWaves x 64 partial sums
    int8_t *key = reinterpret_cast<int8_t *>(smem);
    uint64_t *part = reinterpret_cast<uint64_t *>(smem + ((n + 7) & ~7));
    for (int i = threadIdx.x; i < n; i += blockDim.x) key[i] = s[i];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const LweLane L = lwe_lane(G, C, F, blockIdx.x, lane);
    const int64_t rowlen = (int64_t)n + 1;
    const int64_t q = (L.b * F + L.f) * C + L.c;                     // ciphertext index
    uint64_t *w = ct + (L.b * F + L.f) * rowlen * C + L.c;           // word j at w[j * C]
    // word range of this wave, starting on a multiple of 4 (4-byte key reads)
    const int per = ((n + 4 * kWaves - 1) / (4 * kWaves)) * 4, j0 = wave * per, j1 = min(n, j0 + per);
    uint64_t z = seed_a + ((ct_index0 + (uint64_t)q) * (uint64_t)n + (uint64_t)j0 + 1) * kGamma;
    // <a, s> as (sum over s_j = +1) - (sum over s_j = -1), selected with
    // wave-uniform masks
    uint64_t acc_p = 0, acc_n = 0;
    if (L.ok) {
        int j = j0;
        uint64_t *wj = w + (int64_t)j0 * C;  // word j (stepped: no per-word 64-bit multiply)
        for (; j + 4 <= j1; j += 4) {
            const uint32_t k4 = key4(key, j);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t a = splitmix_mix(z);
                z += kGamma;
                if (STORE_A) *wj = a;
                wj += C;
                acc_p += a & key_mask(k4, k, 1);
                acc_n += a & key_mask(k4, k, -1);
            }
        }
        for (; j < j1; ++j) {
            const uint64_t a = splitmix_mix(z);
            z += kGamma;
            if (STORE_A) *wj = a;
            wj += C;
            const uint32_t k1 = __builtin_amdgcn_readfirstlane((uint32_t)(uint8_t)key[j]);
            acc_p += a & key_mask(k1, 0, 1);
            acc_n += a & key_mask(k1, 0, -1);
        }
    }
    part[wave * 64 + lane] = acc_p - acc_n;
    __syncthreads();
    if (wave == 0 && L.ok) {
        const uint64_t dot = part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane];
        const int64_t mi = (L.b * C + L.c) * F + L.f;
        const uint64_t bword = dot + (uint64_t)(int64_t)e[mi] + delta * (uint64_t)m[mi];
        if (STORE_A)
            w[(int64_t)n * C] = bword;
        else
            ct[(L.b * F + L.f) * C + L.c] = bword;
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

__global__ __launch_bounds__(64 * kDecWaves) void decrypt_kernel(const uint64_t *__restrict__ ct, const int8_t *__restrict__ s,
                                                      int C, int64_t F, int n, uint32_t p, uint32_t *__restrict__ m,
                                                      LweGroups G) {
    extern __shared__ uint8_t smem[];
    int8_t *key = reinterpret_cast<int8_t *>(smem);
    uint64_t *part = reinterpret_cast<uint64_t *>(smem + ((n + 7) & ~7));
    for (int i = threadIdx.x; i < n; i += blockDim.x) key[i] = s[i];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const LweLane L = lwe_lane(G, C, F, blockIdx.x, lane);
    const int64_t rowlen = (int64_t)n + 1;
    const uint64_t *w = ct + (L.b * F + L.f) * rowlen * C + L.c;
    // word range of this wave, starting on a multiple of 4 (4-byte key reads)
    const int per = ((n + 4 * kDecWaves - 1) / (4 * kDecWaves)) * 4, j0 = wave * per, j1 = min(n, j0 + per);
    uint64_t acc_p = 0, acc_n = 0;
    if (L.ok) {
        int j = j0;
        // 16 words per lane in flight at once; the ciphertexts are read once,
        // so the loads are non-temporal (in a step, Dec follows HomConv's
        // write stream: temporal loads cost it a fifth of its time)
        for (; j + 16 <= j1; j += 16) {
            uint64_t x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = __builtin_nontemporal_load(&w[(int64_t)(j + k) * C]);
#pragma unroll
            for (int k4i = 0; k4i < 4; ++k4i) {
                const uint32_t k4 = key4(key, j + 4 * k4i);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    acc_p += x[4 * k4i + k] & key_mask(k4, k, 1);
                    acc_n += x[4 * k4i + k] & key_mask(k4, k, -1);
                }
            }
        }
        for (; j < j1; ++j) {
            const uint64_t x = w[(int64_t)j * C];
            const uint32_t k1 = __builtin_amdgcn_readfirstlane((uint32_t)(uint8_t)key[j]);
            acc_p += x & key_mask(k1, 0, 1);
            acc_n += x & key_mask(k1, 0, -1);
        }
    }
    part[wave * 64 + lane] = acc_p - acc_n;
    __syncthreads();
    if (wave == 0 && L.ok) {
        uint64_t dot = 0;
#pragma unroll
        for (int k = 0; k < kDecWaves; ++k) dot += part[k * 64 + lane];
        m[(L.b * C + L.c) * F + L.f] = decode(w[(int64_t)n * C] - dot, p);
    }
}

// Rounded-Gaussian errors from the public generator: one thread per error
// e[b][c][f] (f fastest, so the int32 stores are contiguous); the generator
// output is number ct_index0 + q + 1 of seed_e for the ciphertext index
// q = (b F + f) C + c; its top bit is the sign, bits 15..62 a uniform
// v < 2^48, and |e| the number of thresholds <= v (binary search over the
// non-decreasing table in LDS).
__global__ __launch_bounds__(256) void sample_errors_kernel(const uint64_t *__restrict__ cdt, uint64_t seed_e,
                                                            uint64_t ct_index0, int64_t B, int C, int64_t F,
                                                            int32_t *__restrict__ e) {
    __shared__ uint64_t T[kCdtSize];
    if (threadIdx.x < kCdtSize) T[threadIdx.x] = cdt[threadIdx.x];
    __syncthreads();
    const int64_t total = B * C * F;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = i % F, bc = i / F, b = bc / C;
        const int c = (int)(bc % C);
        const uint64_t q = (uint64_t)((b * F + f) * C + c);
        const uint64_t u = splitmix_mix(seed_e + (ct_index0 + q + 1) * kGamma);
        const uint64_t v = (u >> 15) & ((1ull << kCdtBits) - 1);
        int lo = 0, hi = kCdtSize;  // the count lies in [lo, hi]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (T[mid] <= v)
                lo = mid + 1;
            else
                hi = mid;
        }
        e[i] = (u >> 63) && lo ? -lo : lo;
    }
}

static int check_lwe(const ensei_ctx *ctx, int64_t B, int C, int64_t F, int n, int64_t *groups) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (B <= 0 || C <= 0 || F <= 0 || n <= 0) return ENSEI_ERR_ARG;
    if (n > ENSEI_MAX_LWE_N) return ENSEI_ERR_LIMIT;
    const LweGroups G = lwe_groups(C, F);
    *groups = B * G.f_groups * G.c_blocks;
    if (*groups > 0x7fffffff) return ENSEI_ERR_LIMIT;
    return ENSEI_OK;
}

}  // namespace ensei

using namespace ensei;

extern "C" {

int ensei_encrypt(ensei_ctx *ctx, const uint32_t *m, const int8_t *s, const int32_t *e, int64_t batch, int C,
                  int64_t F, int n, uint64_t seed_a, uint64_t ct_index0, uint64_t *ct, void *stream) {
    int64_t groups;
    int st = check_lwe(ctx, batch, C, F, n, &groups);
    if (st) return st;
    if (!m || !s || !e || !ct) return ENSEI_ERR_ARG;
    if (((uintptr_t)m & 3) || ((uintptr_t)e & 3) || ((uintptr_t)ct & 7)) return ENSEI_ERR_ALIGN;
    const size_t num = (size_t)batch * C * F, ctb = num * (n + 1) * 8;
    if (overlaps(ct, ctb, m, num * 4) || overlaps(ct, ctb, e, num * 4) || overlaps(ct, ctb, s, (size_t)n))
        return ENSEI_ERR_OVERLAP;
    const size_t smem = ((n + 7) & ~7) + kWaves * 64 * 8;
    hipLaunchKernelGGL(encrypt_kernel<true>, dim3((unsigned)groups), dim3(256), smem, (hipStream_t)stream, m, s, e, C,
                       F, n, seed_a, ct_index0, ctx->delta, ct, lwe_groups(C, F));
    return launch_status();
}

int ensei_encrypt_seeded(ensei_ctx *ctx, const uint32_t *m, const int8_t *s, const int32_t *e, int64_t batch, int C,
                         int64_t F, int n, uint64_t seed_a, uint64_t ct_index0, uint64_t *b_out, void *stream) {
    int64_t groups;
    int st = check_lwe(ctx, batch, C, F, n, &groups);
    if (st) return st;
    if (!m || !s || !e || !b_out) return ENSEI_ERR_ARG;
    if (((uintptr_t)m & 3) || ((uintptr_t)e & 3) || ((uintptr_t)b_out & 7)) return ENSEI_ERR_ALIGN;
    const size_t num = (size_t)batch * C * F;
    if (overlaps(b_out, num * 8, m, num * 4) || overlaps(b_out, num * 8, e, num * 4) ||
        overlaps(b_out, num * 8, s, (size_t)n))
        return ENSEI_ERR_OVERLAP;
    const size_t smem = ((n + 7) & ~7) + kWaves * 64 * 8;
    hipLaunchKernelGGL(encrypt_kernel<false>, dim3((unsigned)groups), dim3(256), smem, (hipStream_t)stream, m, s, e, C,
                       F, n, seed_a, ct_index0, ctx->delta, b_out, lwe_groups(C, F));
    return launch_status();
}

int ensei_sample_errors(ensei_ctx *ctx, uint64_t seed_e, uint64_t ct_index0, int64_t batch, int C, int64_t F,
                        int32_t *e, void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!e || batch <= 0 || C <= 0 || F <= 0) return ENSEI_ERR_ARG;
    if (batch > ((int64_t)1 << 40) / C / F) return ENSEI_ERR_LIMIT;
    if ((uintptr_t)e & 3) return ENSEI_ERR_ALIGN;
    const int64_t total = batch * C * F, blocks = (total + 255) / 256;
    hipLaunchKernelGGL(sample_errors_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                       (hipStream_t)stream, ctx->d_cdt, seed_e, ct_index0, batch, C, F, e);
    return launch_status();
}

int ensei_decrypt(ensei_ctx *ctx, const uint64_t *ct, const int8_t *s, int64_t batch, int C, int64_t F, int n,
                  uint32_t *m, void *stream) {
    int64_t groups;
    int st = check_lwe(ctx, batch, C, F, n, &groups);
    if (st) return st;
    if (!m || !s || !ct) return ENSEI_ERR_ARG;
    if (((uintptr_t)m & 3) || ((uintptr_t)ct & 7)) return ENSEI_ERR_ALIGN;
    const size_t num = (size_t)batch * C * F, ctb = num * (n + 1) * 8;
    if (overlaps(m, num * 4, ct, ctb) || overlaps(m, num * 4, s, (size_t)n)) return ENSEI_ERR_OVERLAP;
    const size_t smem = ((n + 7) & ~7) + kDecWaves * 64 * 8;
    hipLaunchKernelGGL(decrypt_kernel, dim3((unsigned)groups), dim3(64 * kDecWaves), smem, (hipStream_t)stream, ct, s, C, F, n,
                       ctx->p, m, lwe_groups(C, F));
    return launch_status();
}

}  // extern "C"
