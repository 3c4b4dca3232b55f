// The packed (BFV / RLWE) instantiation: negacyclic transforms over three
// primes below 2^30 (t, q0, q1), encryption in evaluation form with the
// public a^ generated in registers, SIMDScMult with the channel sum and the
// masks, CRT decryption with exact rounding, and the fold of slot blocks.
//
// Every polynomial transform runs in one 256-thread workgroup over an n-word
// LDS array: Cooley-Tukey (forward, natural in, bit-reversed out) and
// Gentleman-Sande (inverse, bit-reversed in, natural out) butterflies with
// the merged psi powers in bit-reversed order, Shoup multiplications by
// precomputed companions; residues enter and leave a transform in [0, m)
// (inside it they stay lazily reduced). The layouts at the ABI are natural
// slot order; the bit reversal happens on the LDS reads.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/ensei_bfv.h"
#include "ensei_internal.hpp"

namespace {

constexpr int kNT = 256;          // threads per polynomial
constexpr int kMaxN = 4096;       // ring degree limit (a polynomial's LDS array: 4 n bytes)
constexpr int kPer = kMaxN / kNT; // coefficients per thread at most
constexpr int kMods = 3;          // t, q0, q1

// Per modulus: m, n^-1 and its companion.
struct Mod {
    uint32_t m, ninv, ninv_sh;
};

// What the kernels need of a context, passed by value.
struct BfvK {
    Mod md[kMods];
    uint32_t delta[2], delta_sh[2];   // Delta = round(q / t), mod q_l, and companion
    uint32_t r32[2], r32_sh[2];       // 2^32 mod q_l and companion (64-bit reduction)
    uint32_t mont[2];                 // -q_l^-1 mod 2^32 (Montgomery reduction)
    uint32_t one_sh[3];               // floor(2^32 / m): reduces a 32-bit word mod m
    uint32_t q0inv, q0inv_sh;         // q0^-1 mod q1 and companion
    uint32_t t;
    int n, logn;
    uint64_t q;                       // q0 q1
    uint64_t half_q;                  // (q - 1) / 2
    double inv_q;                     // 1 / q
    const uint32_t *tw;               // [3 moduli][4][n]: fwd w, fwd w', inv w, inv w' (bit-reversed order)
};

__device__ __forceinline__ uint32_t red1(uint32_t x, uint32_t m) {
    // x in [0, 2m) -> [0, m): x - m wraps above x when x < m
    const uint32_t y = x - m;
    return y < x ? y : x;
}

// x * w mod m in [0, m) for any 32-bit x, w < m < 2^30, wsh = floor(w 2^32 / m)
__device__ __forceinline__ uint32_t mulsh(uint32_t x, uint32_t w, uint32_t wsh, uint32_t m) {
    const uint32_t qt = __umulhi(x, wsh);
    return red1(x * w - qt * m, m);
}

// Shoup's product without its final correction: x w mod m + {0, m}, in
// [0, 2m), for any 32-bit x
__device__ __forceinline__ uint32_t mulsh_lazy(uint32_t x, uint32_t w, uint32_t wsh, uint32_t m) {
    return x * w - __umulhi(x, wsh) * m;
}

__device__ __forceinline__ uint32_t addm(uint32_t a, uint32_t b, uint32_t m) { return red1(a + b, m); }
__device__ __forceinline__ uint32_t subm(uint32_t a, uint32_t b, uint32_t m) { return red1(a + m - b, m); }

// x mod m for a 64-bit x: hi * (2^32 mod m) + lo, each reduced
__device__ __forceinline__ uint32_t mod64(uint64_t x, uint32_t m, uint32_t r32, uint32_t r32_sh, uint32_t one_sh) {
    const uint32_t h = mulsh((uint32_t)(x >> 32), r32, r32_sh, m);
    const uint32_t l = mulsh((uint32_t)x, 1u, one_sh, m);
    return addm(h, l, m);
}

constexpr uint64_t kSplitGamma = 0x9e3779b97f4a7c15ULL;

// SplitMix64's output for the state z = seed + k gamma (the generator's
// finaliser; splitmix64(seed, k) below)
__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * kSplitGamma;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// A kernel's LDS (dynamic, sized at launch for the context's n): arrays of
// n words one after another, a[w] the w-th
extern __shared__ __attribute__((aligned(16))) uint32_t bfv_lds[];
struct LdsArrays {
    uint32_t *p;
    int n;
    __device__ uint32_t *operator[](int w) const { return p + w * n; }
};

__device__ __forceinline__ int brev(int x, int logn) { return (int)(__brev((uint32_t)x) >> (32 - logn)); }

// In-place transform of a[0..n) in LDS mod md.m; modulus index mi selects
// the twiddles. Forward: natural in, out[i] = u(psi^(2 brev(i) + 1)).
// Inverse: in[i] = slot brev(i), natural coefficients out, times n^-1.
// Forward stage s (0 <= s < logn) pairs j and j + t, t = n >> (s + 1), with
// twiddle 2^s + j / 2t; inverse stage s pairs j and j + t, t = 2^s, with
// twiddle (n >> (s + 1)) + j / 2t. The stages are taken up to three at a
// time: a thread loads the 2^R elements j0 + k stride of one unit (one
// radix-2^R sub-transform) into registers, applies the R stages there and
// writes them back, so a transform needs ceil(logn / 3) barriers, not logn.
// The butterflies are Harvey's lazy ones (m < 2^30, so 4m fits 32 bits):
// forward values stay in [0, 4m), inverse ones in [0, 2m), and the last
// pass reduces them to [0, m).
// na arrays a + v n (v < na) are transformed together, sharing them;
// array v under modulus index mi + v mstep (the same modulus, or one limb
// per array). JA > 1: groups of JA arrays of one modulus (mstep = 0) go
// through a thread together, which reads each twiddle once for all of them.
template <bool INV, int JA = 1>
__device__ void ntt_lds(uint32_t *a, const BfvK &K, int mi, int na = JA, int mstep = 0) {
    const int n = K.n, logn = K.logn, tid = threadIdx.x;
    // stages s0 .. s0 + R - 1; LAST: the transform's last pass (forward:
    // reduce to [0, m); inverse: multiply by n^-1, which also reduces)
    auto group = [&](auto r_tag, int s0, bool last) {
        constexpr int R = decltype(r_tag)::value, E = 1 << R;
        // log2 of the unit's stride: the group's smallest t
        const int ls = INV ? s0 : logn - s0 - R;
        // item w: unit u of arrays v0 .. v0 + JA - 1 (JA > 1: one modulus,
        // each twiddle read once for all of them)
        for (int w = tid; w < ((na / JA) << (logn - R)); w += kNT) {
            const int v0 = (w >> (logn - R)) * JA, mv = mi + v0 * mstep;
            uint32_t *const av = a + v0 * n;
            const int u = w & ((n >> R) - 1);
            const uint32_t m = K.md[mv].m;
            const uint32_t *tw = K.tw + (size_t)mv * 4 * n + (INV ? 2 * n : 0);
            const uint32_t *tws = tw + n;
            const int blk = u >> ls, j0 = (blk << (ls + R)) + (u & ((1 << ls) - 1));
            uint32_t x[JA][E];
#pragma unroll
            for (int q = 0; q < JA; ++q)
#pragma unroll
                for (int k = 0; k < E; ++k) x[q][k] = av[q * n + j0 + (k << ls)];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int st = s0 + r;
                const int d = INV ? 1 << r : 1 << (R - 1 - r);  // t / stride
                const int base = INV ? n >> (st + 1) : 1 << st;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if (k & d) continue;
                    // (j0 + k stride) / 2t: the butterflies of a unit share
                    // one twiddle in the group's first stage, 2^R / 2 in its last
                    const int i = INV ? (blk << (R - 1 - r)) + (k >> (r + 1)) : (blk << r) + (k >> (R - r));
                    const uint32_t S = __ldg(tw + base + i), Ssh = __ldg(tws + base + i);
#pragma unroll
                    for (int q = 0; q < JA; ++q) {
                        if (!INV) {
                            // inputs in [0, 4m)
                            const uint32_t U = red1(x[q][k], 2 * m);                // [0, 2m)
                            const uint32_t V = mulsh_lazy(x[q][k + d], S, Ssh, m);  // [0, 2m)
                            x[q][k] = U + V;                                        // [0, 4m)
                            x[q][k + d] = U - V + 2 * m;                            // (0, 4m)
                        } else {
                            // inputs in [0, 2m)
                            const uint32_t U = x[q][k], V = x[q][k + d];
                            x[q][k] = red1(U + V, 2 * m);                           // [0, 2m)
                            x[q][k + d] = mulsh_lazy(U - V + 2 * m, S, Ssh, m);     // [0, 2m)
                        }
                    }
                }
            }
            if (last) {
#pragma unroll
                for (int q = 0; q < JA; ++q)
#pragma unroll
                    for (int k = 0; k < E; ++k)
                        x[q][k] = INV ? mulsh(x[q][k], K.md[mv].ninv, K.md[mv].ninv_sh, m)
                                      : red1(red1(x[q][k], 2 * m), m);
            }
#pragma unroll
            for (int q = 0; q < JA; ++q)
#pragma unroll
                for (int k = 0; k < E; ++k) av[q * n + j0 + (k << ls)] = x[q][k];
        }
        __syncthreads();
    };
    int s = 0;
    for (; s + 3 <= logn; s += 3) group(std::integral_constant<int, 3>{}, s, s + 3 == logn);
    if (logn - s == 2)
        group(std::integral_constant<int, 2>{}, s, true);
    else if (logn - s == 1)
        group(std::integral_constant<int, 1>{}, s, true);
}

// Slot s of packed vector (b, g, k) of a [B][C][F] spectrum array: channel
// g P + j, frequency k Fp + s mod Fp (Fp = min(F, n)); 0 past the channels.
__device__ __forceinline__ uint32_t packed_slot(const uint32_t *x, int64_t b, int C, int64_t F, int P, int Fp, int g,
                                                int k, int s) {
    const int j = s / Fp, c = g * P + j;
    if (c >= C) return 0;
    return x[((int64_t)b * C + c) * F + (int64_t)k * Fp + (s - j * Fp)];
}

// Enc of packed vector ci (one workgroup each): slots -> INTT_t -> per limb
// Delta u + e -> NTT_q -> b^ = a^ s^ + that, a^ from the generator.
__global__ __launch_bounds__(kNT) void bfv_encrypt_kernel(BfvK K, const uint32_t *__restrict__ x, int C, int64_t F,
                                                          int P, int Fp, int G, int KC,
                                                          const uint32_t *__restrict__ s_hat,
                                                          const int32_t *__restrict__ e, uint64_t seed_a,
                                                          uint64_t ct_index0, uint32_t *__restrict__ ct) {
    const int n = K.n, tid = threadIdx.x;
    const LdsArrays a{bfv_lds, n};  // one array per limb
    const int64_t ci = blockIdx.x;
    const int64_t b = ci / ((int64_t)G * KC);
    const int rest = (int)(ci - b * G * KC), g = rest / KC, k = rest - g * KC;
    for (int s = tid; s < n; s += kNT) a[0][brev(s, K.logn)] = packed_slot(x, b, C, F, P, Fp, g, k, s);
    __syncthreads();
    ntt_lds<true>(a[0], K, 0);  // u = INTT_t(slots), natural order
    uint32_t u[kPer];
    int32_t ev[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int s = tid + r * kNT;
        if (s < n) {
            u[r] = a[0][s];
            ev[r] = e[ci * n + s];
        }
    }
    __syncthreads();
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = K.md[1 + l].m;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int s = tid + r * kNT;
            if (s < n) {
                const uint32_t em = ev[r] < 0 ? m - mulsh((uint32_t)(-ev[r]), 1u, K.one_sh[1 + l], m)
                                              : mulsh((uint32_t)ev[r], 1u, K.one_sh[1 + l], m);
                a[l][s] = red1(mulsh(u[r], K.delta[l], K.delta_sh[l], m) + red1(em, m), m);
            }
        }
    }
    __syncthreads();
    ntt_lds<false>(a[0], K, 1, 2, 1);  // both limbs
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = K.md[1 + l].m;
        uint32_t *wa = ct + ((ci * 2 + l) * 2) * (int64_t)n, *wb = wa + n;
        const uint32_t *sh = s_hat + (size_t)l * 2 * n;
        for (int s = tid; s < n; s += kNT) {
            const uint64_t z = splitmix64(seed_a, ((ct_index0 + (uint64_t)ci) * 2 + (uint64_t)l) * (uint64_t)n +
                                                      (uint64_t)s + 1);
            const uint32_t av = mod64(z, m, K.r32[l], K.r32_sh[l], K.one_sh[1 + l]);
            wa[s] = av;
            wb[s] = addm(mulsh(av, sh[s], sh[n + s], m), a[l][brev(s, K.logn)], m);
        }
    }
}

// Plaintext encodings (one workgroup per slot vector):
//   MODE 0 filters: slots gathered from W^ [Cout][Cin][F] for vector (o, g, k),
//          coefficients lifted to (-t/2, t/2], out [..][l][2][n] with companions;
//   MODE 1 masks: slots r[v][n], coefficients scaled by Delta, out [..][l][n];
//   MODE 2 key: coefficients s (int8) directly, out [l][2][n] with companions.
template <int MODE>
__global__ __launch_bounds__(kNT) void bfv_encode_kernel(BfvK K, const void *__restrict__ src, int C, int64_t F, int P,
                                                         int Fp, int G, int KC, uint32_t *__restrict__ out) {
    const int n = K.n, tid = threadIdx.x;
    const LdsArrays a{bfv_lds, n};  // one array per limb
    const int64_t vi = blockIdx.x;
    uint32_t u[kPer];
    int sgn[kPer];
    if (MODE == 2) {
        const int8_t *s8 = static_cast<const int8_t *>(src);
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int s = tid + r * kNT;
            if (s < n) sgn[r] = s8[s];
        }
    } else {
        const uint32_t *x = static_cast<const uint32_t *>(src);
        if (MODE == 0) {
            const int64_t o = vi / ((int64_t)G * KC);
            const int rest = (int)(vi - o * G * KC), g = rest / KC, k = rest - g * KC;
            for (int s = tid; s < n; s += kNT) a[0][brev(s, K.logn)] = packed_slot(x, o, C, F, P, Fp, g, k, s);
        } else {
            for (int s = tid; s < n; s += kNT) a[0][brev(s, K.logn)] = x[vi * n + s];
        }
        __syncthreads();
        ntt_lds<true>(a[0], K, 0);
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int s = tid + r * kNT;
            if (s < n) u[r] = a[0][s];
        }
    }
    __syncthreads();
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = K.md[1 + l].m;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int s = tid + r * kNT;
            if (s >= n) continue;
            uint32_t v;
            if (MODE == 0)
                v = u[r] > K.t / 2 ? u[r] + (m - K.t) : u[r];  // centred lift of u - t
            else if (MODE == 1)
                v = mulsh(u[r], K.delta[l], K.delta_sh[l], m);
            else
                v = sgn[r] < 0 ? m - 1 : (uint32_t)sgn[r];
            a[l][s] = v;
        }
    }
    __syncthreads();
    ntt_lds<false>(a[0], K, 1, 2, 1);  // both limbs
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = K.md[1 + l].m;
        if (MODE == 1) {
            uint32_t *o = out + (vi * 2 + l) * (int64_t)n;
            for (int s = tid; s < n; s += kNT) o[s] = a[l][brev(s, K.logn)];
        } else {
            uint32_t *o = out + (vi * 2 + l) * 2 * (int64_t)n;
            for (int s = tid; s < n; s += kNT) {
                const uint32_t w = a[l][brev(s, K.logn)];
                o[s] = w;
                o[n + s] = (uint32_t)(((uint64_t)w << 32) / m);
            }
        }
    }
}

// SIMDScMult, the sum over input vectors and the masks. One thread per slot
// s of one (chunk k, limb l), kOB outputs x kBB images of both words in
// registers; the filters and inputs of a g are read once per thread. From
// three input vectors on, the products w x < 2^60 are summed exactly in 64
// bits (one multiply-add each), 16 at a time, and reduced mod m once per 16
// input vectors; with one or two, each product is reduced by Shoup's method
// (the 64-bit reduction costs more than two of those).
constexpr int kOB = 4, kBB = 4;
constexpr int kLazyTerms = 16;  // 16 (2^30 - 1)^2 < 2^64
constexpr int kLazyMinG = 3;

__global__ __launch_bounds__(kNT) void bfv_homconv_kernel(BfvK K, const uint32_t *__restrict__ ct_in,
                                                          const uint32_t *__restrict__ w_enc,
                                                          const uint32_t *__restrict__ mask_enc, int64_t B, int G,
                                                          int Cout, int KC, uint32_t *__restrict__ ct_out) {
    const int n = K.n;
    int64_t t = blockIdx.x;
    const int sb = (n + kNT - 1) / kNT;
    const int s = (int)(t % sb) * kNT + threadIdx.x;
    t /= sb;
    const int l = (int)(t % 2);
    t /= 2;
    const int k = (int)(t % KC);
    t /= KC;
    const int nob = (Cout + kOB - 1) / kOB;
    const int o0 = (int)(t % nob) * kOB;
    const int64_t b0 = (t / nob) * kBB;
    const uint32_t m = K.md[1 + l].m;
    if (s >= n) return;
    uint32_t acc[kOB][kBB][2];  // reduced sums
#pragma unroll
    for (int i = 0; i < kOB; ++i)
#pragma unroll
        for (int j = 0; j < kBB; ++j) acc[i][j][0] = acc[i][j][1] = 0;
    for (int g = 0; G < kLazyMinG && g < G; ++g) {
        uint32_t w[kOB], wsh[kOB], x[kBB][2];
#pragma unroll
        for (int i = 0; i < kOB; ++i) {
            const int o = o0 + i < Cout ? o0 + i : Cout - 1;
            const uint32_t *p = w_enc + ((((int64_t)o * G + g) * KC + k) * 2 + l) * 2 * (int64_t)n;
            w[i] = p[s];
            wsh[i] = p[n + s];
        }
#pragma unroll
        for (int j = 0; j < kBB; ++j) {
            const int64_t b = b0 + j < B ? b0 + j : B - 1;
            const uint32_t *p = ct_in + ((((b * G + g) * KC + k) * 2 + l) * 2) * (int64_t)n;
            x[j][0] = p[s];
            x[j][1] = p[n + s];
        }
#pragma unroll
        for (int i = 0; i < kOB; ++i)
#pragma unroll
            for (int j = 0; j < kBB; ++j) {
                acc[i][j][0] = addm(acc[i][j][0], mulsh(x[j][0], w[i], wsh[i], m), m);
                acc[i][j][1] = addm(acc[i][j][1], mulsh(x[j][1], w[i], wsh[i], m), m);
            }
    }
    for (int g0 = 0; G >= kLazyMinG && g0 < G; g0 += kLazyTerms) {
        const int g1 = G - g0 < kLazyTerms ? G : g0 + kLazyTerms;
        uint64_t sum[kOB][kBB][2];  // exact sums of at most kLazyTerms products
#pragma unroll
        for (int i = 0; i < kOB; ++i)
#pragma unroll
            for (int j = 0; j < kBB; ++j) sum[i][j][0] = sum[i][j][1] = 0;
        for (int g = g0; g < g1; ++g) {
            uint32_t w[kOB], x[kBB][2];
#pragma unroll
            for (int i = 0; i < kOB; ++i) {
                const int o = o0 + i < Cout ? o0 + i : Cout - 1;
                w[i] = w_enc[((((int64_t)o * G + g) * KC + k) * 2 + l) * 2 * (int64_t)n + s];
            }
#pragma unroll
            for (int j = 0; j < kBB; ++j) {
                const int64_t b = b0 + j < B ? b0 + j : B - 1;
                const uint32_t *p = ct_in + ((((b * G + g) * KC + k) * 2 + l) * 2) * (int64_t)n;
                x[j][0] = p[s];
                x[j][1] = p[n + s];
            }
#pragma unroll
            for (int i = 0; i < kOB; ++i)
#pragma unroll
                for (int j = 0; j < kBB; ++j) {
                    sum[i][j][0] += (uint64_t)x[j][0] * w[i];
                    sum[i][j][1] += (uint64_t)x[j][1] * w[i];
                }
        }
#pragma unroll
        for (int i = 0; i < kOB; ++i)
#pragma unroll
            for (int j = 0; j < kBB; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    acc[i][j][h] = addm(acc[i][j][h], mod64(sum[i][j][h], m, K.r32[l], K.r32_sh[l], K.one_sh[1 + l]), m);
    }
#pragma unroll
    for (int i = 0; i < kOB; ++i) {
        const int o = o0 + i;
        if (o >= Cout) break;
#pragma unroll
        for (int j = 0; j < kBB; ++j) {
            const int64_t b = b0 + j;
            if (b >= B) break;
            const int64_t vo = (b * Cout + o) * KC + k;
            uint32_t *p = ct_out + ((vo * 2 + l) * 2) * (int64_t)n;
            p[s] = acc[i][j][0];
            p[n + s] = addm(acc[i][j][1], mask_enc[(vo * 2 + l) * (int64_t)n + s], m);
        }
    }
}

// 128-bit values as (hi, lo) pairs of 64-bit words
struct U128 {
    uint64_t hi, lo;
};
__device__ __forceinline__ U128 mul64(uint64_t a, uint64_t b) { return U128{__umul64hi(a, b), a * b}; }
__device__ __forceinline__ U128 add64(U128 x, uint64_t y) {
    const uint64_t lo = x.lo + y;
    return U128{x.hi + (lo < y), lo};
}
__device__ __forceinline__ bool less(U128 x, U128 y) { return x.hi < y.hi || (x.hi == y.hi && x.lo < y.lo); }

// floor((t phi + (q-1)/2) / q) mod t for phi < q: an estimate in double
// (within one of the quotient), made exact by comparing est q with the
// numerator in 128-bit integers.
__device__ __forceinline__ uint32_t round_tq(uint64_t phi, const BfvK &K) {
    const U128 num = add64(mul64(phi, K.t), K.half_q);
    uint64_t est = (uint64_t)((double)phi * ((double)K.t * K.inv_q) + 0.5);
    while (est > 0 && less(num, mul64(est, K.q))) --est;          // est q <= num
    while (!less(num, mul64(est + 1, K.q))) ++est;                // num < (est + 1) q
    return est >= K.t ? (uint32_t)(est - K.t) : (uint32_t)est;   // est <= t
}

// Dec of ciphertext ci (one workgroup each): per limb b^ - a^ s^ -> INTT_q,
// CRT to [0, q), round(t phi / q) mod t, NTT_t -> natural slots.
__global__ __launch_bounds__(kNT) void bfv_decrypt_kernel(BfvK K, const uint32_t *__restrict__ ct,
                                                          const uint32_t *__restrict__ s_hat,
                                                          uint32_t *__restrict__ v) {
    const int n = K.n, tid = threadIdx.x;
    uint32_t *const a = bfv_lds;
    const int64_t ci = blockIdx.x;
    uint32_t r0[kPer];
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = K.md[1 + l].m;
        const uint32_t *wa = ct + ((ci * 2 + l) * 2) * (int64_t)n, *wb = wa + n;
        const uint32_t *sh = s_hat + (size_t)l * 2 * n;
        if (l) __syncthreads();
        for (int s = tid; s < n; s += kNT) a[brev(s, K.logn)] = subm(wb[s], mulsh(wa[s], sh[s], sh[n + s], m), m);
        __syncthreads();
        ntt_lds<true>(a, K, 1 + l);
        if (l == 0) {
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int s = tid + r * kNT;
                if (s < n) r0[r] = a[s];
            }
        }
    }
    // a holds the limb-1 residues; join and round in place (each thread its own coefficients)
    const uint32_t q0 = K.md[1].m, q1 = K.md[2].m;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int s = tid + r * kNT;
        if (s >= n) continue;
        const uint32_t x0 = r0[r], x1 = a[s];
        const uint32_t x0m = mulsh(x0, 1u, K.one_sh[2], q1);  // x0 mod q1
        const uint32_t h = mulsh(subm(x1, x0m, q1), K.q0inv, K.q0inv_sh, q1);
        const uint64_t phi = (uint64_t)x0 + (uint64_t)q0 * h;  // < q
        a[s] = round_tq(phi, K);
    }
    __syncthreads();
    ntt_lds<false>(a, K, 0);
    for (int s = tid; s < n; s += kNT) v[ci * n + s] = a[brev(s, K.logn)];
}

// Circuit privacy: ciphertext ci gains a fresh public-key encryption of zero,
// (a^_pk rho^ + e1^, b^_pk rho^ + e2^). The draws (coefficient domain) come
// from the generator by multiply-shift and are transformed per limb.
constexpr uint32_t kE1Bound = 16;

// draw number k in [-bound, bound] from the generator's state z = seed + k gamma
__device__ __forceinline__ int32_t draw_at(uint64_t z, uint32_t bound) {
    const uint64_t x = splitmix_out(z);
    return (int32_t)((int64_t)(((x >> 32) * (2 * (uint64_t)bound + 1)) >> 32) - (int64_t)bound);
}

// x R^-1 mod m (R = 2^32) for x < m 2^32, with mont = -m^-1 mod 2^32
// (Montgomery's reduction: x + (x mont mod R) m is divisible by R)
__device__ __forceinline__ uint32_t redc(uint64_t x, uint32_t m, uint32_t mont) {
    const uint32_t t = (uint32_t)x * mont;
    return red1((uint32_t)((x + (uint64_t)t * m) >> 32), m);
}

__global__ __launch_bounds__(kNT) void bfv_rerandomize_kernel(BfvK K, uint32_t *__restrict__ ct,
                                                              const uint32_t *__restrict__ pk, uint64_t seed_r,
                                                              uint64_t ct_index0, uint32_t flood) {
    const int n = K.n, tid = threadIdx.x;
    const LdsArrays a{bfv_lds, n};  // the three draws
    const int64_t ci = blockIdx.x;
    // draw k = ((ct_index0 + ci) 3 + w) n + s + 1 of the generator seeded with
    // seed_r: its state seed_r + k gamma stepped by n gamma per w and kNT gamma
    // per r
    int32_t d[3][kPer];
    const uint64_t z0 = seed_r + (((ct_index0 + (uint64_t)ci) * 3) * (uint64_t)n + (uint64_t)tid + 1) * kSplitGamma;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        const uint32_t bound = w == 0 ? 1u : w == 1 ? kE1Bound : flood;
        uint64_t z = z0 + (uint64_t)w * (uint64_t)n * kSplitGamma;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int s = tid + r * kNT;
            if (s < n) d[w][r] = draw_at(z, bound);
            z += (uint64_t)kNT * kSplitGamma;
        }
    }
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = K.md[1 + l].m;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int s = tid + r * kNT;
                if (s < n) {
                    const int32_t v = d[w][r];
                    if (w == 0) {
                        // rho in {-1, 0, 1}, times R = 2^32 (Montgomery form for
                        // the products below)
                        a[w][s] = v == 0 ? 0u : v > 0 ? K.r32[l] : m - K.r32[l];
                    } else {
                        const uint32_t mag = mulsh((uint32_t)(v < 0 ? -v : v), 1u, K.one_sh[1 + l], m);
                        a[w][s] = v < 0 ? red1(m - mag, m) : mag;
                    }
                }
            }
        __syncthreads();
        ntt_lds<false, 3>(a[0], K, 1 + l);  // the three draws together, one twiddle read for the three
        uint32_t *wa = ct + ((ci * 2 + l) * 2) * (int64_t)n, *wb = wa + n;
        const uint32_t *pa = pk + (size_t)l * 2 * n, *pb = pa + n;
        for (int s = tid; s < n; s += kNT) {
            const int i = brev(s, K.logn);
            const uint32_t rho = a[0][i];  // NTT(rho) R mod m
            const uint32_t ta = redc((uint64_t)pa[s] * rho, m, K.mont[l]);
            const uint32_t tb = redc((uint64_t)pb[s] * rho, m, K.mont[l]);
            wa[s] = addm(addm(wa[s], ta, m), a[1][i], m);
            wb[s] = addm(addm(wb[s], tb, m), a[2][i], m);
        }
    }
}

// The fold: y[b][c][f] = (+/-) sum of the slot blocks holding (c, f), mod t.
__global__ __launch_bounds__(256) void bfv_fold_kernel(const uint32_t *__restrict__ v, int64_t B, int C, int64_t F,
                                                       int n, int P, int Fp, int KC, uint32_t t, uint32_t t_sh,
                                                       int negate, uint32_t *__restrict__ y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * C * F) return;
    const int64_t f = idx % F, bc = idx / F;
    const int k = (int)(f / Fp), fr = (int)(f - (int64_t)k * Fp);
    const uint32_t *p = v + (bc * KC + k) * (int64_t)n + fr;
    uint32_t acc = 0;
    for (int j = 0; j < P; ++j) acc = addm(acc, mulsh(p[j * Fp], 1u, t_sh, t), t);
    y[idx] = negate && acc ? t - acc : acc;
}

// ------------------------------------------------------------- host side --

uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }
uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = h_mulmod(r, a, m);
        a = h_mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}
bool h_is_prime(uint64_t m) {
    if (m < 2) return false;
    for (uint64_t d = 2; d * d <= m; ++d)
        if (m % d == 0) return false;
    return true;
}
uint64_t h_generator(uint64_t m) {
    uint64_t r = m - 1, fac[64];
    int nf = 0;
    for (uint64_t d = 2; d * d <= r; ++d)
        if (r % d == 0) {
            fac[nf++] = d;
            while (r % d == 0) r /= d;
        }
    if (r > 1) fac[nf++] = r;
    for (uint64_t g = 2; g < m; ++g) {
        bool ok = true;
        for (int i = 0; i < nf && ok; ++i) ok = h_powmod(g, (m - 1) / fac[i], m) != 1;
        if (ok) return g;
    }
    return 0;
}
uint32_t companion(uint32_t w, uint32_t m) { return (uint32_t)(((uint64_t)w << 32) / m); }
int h_brev(int x, int logn) {
    int r = 0;
    for (int i = 0; i < logn; ++i) r |= ((x >> i) & 1) << (logn - 1 - i);
    return r;
}

struct Geometry {
    int P, Fp, G, KC;
};

bool geometry(int n, int C, int64_t F, Geometry *gm) {
    if (C <= 0 || F <= 0 || (F & (F - 1))) return false;
    if (F <= n) {
        gm->P = (int)(n / F);
        gm->Fp = (int)F;
        gm->KC = 1;
    } else {
        gm->P = 1;
        gm->Fp = n;
        gm->KC = (int)(F / n);
    }
    gm->G = (C + gm->P - 1) / gm->P;
    return true;
}

}  // namespace

struct ensei_bfv_ctx {
    int device = 0;
    BfvK K;
    uint32_t *d_tw = nullptr;
};

namespace {

// dynamic LDS of a kernel holding `arrays` polynomials of the context's n words
size_t lds_bytes(const ensei_bfv_ctx *ctx, int arrays) { return (size_t)arrays * ctx->K.n * sizeof(uint32_t); }

int check_bfv(const ensei_bfv_ctx *ctx) {
    if (!ctx) return ENSEI_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ENSEI_ERR_HIP;
    return dev == ctx->device ? ENSEI_OK : ENSEI_ERR_DEVICE;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3) == 0; }

}  // namespace

extern "C" {

int ensei_bfv_ctx_create(ensei_bfv_ctx **out, uint32_t t, uint32_t q0, uint32_t q1, int n, int device) {
    if (!out) return ENSEI_ERR_ARG;
    *out = nullptr;
    const int logn = ensei::ilog2_pow2(n);
    if (logn < 4 || n > kMaxN) return ENSEI_ERR_ARG;
    const uint32_t mods[kMods] = {t, q0, q1};
    for (int i = 0; i < kMods; ++i) {
        const uint32_t m = mods[i];
        if (m < 3 || m >= (1u << 30) || !h_is_prime(m) || (m - 1) % (2u * (uint32_t)n) != 0) return ENSEI_ERR_MODULUS;
    }
    if (t == q0 || t == q1 || q0 == q1) return ENSEI_ERR_MODULUS;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return ENSEI_ERR_HIP;
    if (device < 0 || device >= ndev) return ENSEI_ERR_ARG;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return ENSEI_ERR_HIP;
    ensei_bfv_ctx *c = new ensei_bfv_ctx;
    c->device = device;
    BfvK &K = c->K;
    K.n = n;
    K.logn = logn;
    K.t = t;
    std::vector<uint32_t> tw((size_t)kMods * 4 * n);
    for (int i = 0; i < kMods; ++i) {
        const uint32_t m = mods[i];
        const uint64_t psi = h_powmod(h_generator(m), (m - 1) / (2 * (uint64_t)n), m);
        const uint64_t psi_inv = h_powmod(psi, m - 2, m);
        uint32_t *T = tw.data() + (size_t)i * 4 * n;
        for (int k = 0; k < n; ++k) {
            const int e = h_brev(k, logn);
            T[k] = (uint32_t)h_powmod(psi, e, m);
            T[n + k] = companion(T[k], m);
            T[2 * n + k] = (uint32_t)h_powmod(psi_inv, e, m);
            T[3 * n + k] = companion(T[2 * n + k], m);
        }
        K.md[i].m = m;
        K.md[i].ninv = (uint32_t)h_powmod(n, m - 2, m);
        K.md[i].ninv_sh = companion(K.md[i].ninv, m);
        K.one_sh[i] = companion(1, m);
    }
    const unsigned __int128 q = (unsigned __int128)q0 * q1;
    const unsigned __int128 delta = (q + t / 2) / t;  // nearest integer to q / t (t odd)
    for (int l = 0; l < 2; ++l) {
        const uint32_t m = mods[1 + l];
        K.delta[l] = (uint32_t)(delta % m);
        K.delta_sh[l] = companion(K.delta[l], m);
        K.r32[l] = (uint32_t)((((uint64_t)1) << 32) % m);
        K.r32_sh[l] = companion(K.r32[l], m);
        uint32_t inv = m;  // m^-1 mod 2^32 by Newton's iteration (m odd: correct to 3 bits, doubling)
        for (int it = 0; it < 5; ++it) inv *= 2u - m * inv;
        K.mont[l] = 0u - inv;
    }
    K.q0inv = (uint32_t)h_powmod(q0 % q1, q1 - 2, q1);
    K.q0inv_sh = companion(K.q0inv, q1);
    K.q = (uint64_t)q;
    K.half_q = (uint64_t)((q - 1) / 2);
    K.inv_q = 1.0 / (double)K.q;
    bool ok = hipMalloc(&c->d_tw, tw.size() * 4) == hipSuccess;
    if (!ok) c->d_tw = nullptr;
    ok = ok && hipMemcpy(c->d_tw, tw.data(), tw.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    K.tw = c->d_tw;
    (void)hipSetDevice(prev);
    if (!ok) {
        if (c->d_tw) (void)hipFree(c->d_tw);
        delete c;
        return ENSEI_ERR_HIP;
    }
    *out = c;
    return ENSEI_OK;
}

int ensei_bfv_ctx_destroy(ensei_bfv_ctx *ctx) {
    if (!ctx) return ENSEI_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    if (ctx->d_tw) (void)hipFree(ctx->d_tw);
    (void)hipSetDevice(prev);
    delete ctx;
    return ENSEI_OK;
}

int64_t ensei_bfv_vectors(const ensei_bfv_ctx *ctx, int C, int64_t F) {
    Geometry gm;
    if (!ctx || !geometry(ctx->K.n, C, F, &gm)) return 0;
    return (int64_t)gm.G * gm.KC;
}

int ensei_bfv_key(ensei_bfv_ctx *ctx, const int8_t *s, uint32_t *s_hat, void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!s || !s_hat) return ENSEI_ERR_ARG;
    if (!aligned4(s_hat)) return ENSEI_ERR_ALIGN;
    const int n = ctx->K.n;
    if (ensei::overlaps(s_hat, (size_t)4 * n * 4, s, n)) return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(bfv_encode_kernel<2>, dim3(1), dim3(kNT), lds_bytes(ctx, 2), (hipStream_t)stream, ctx->K, s, 1, (int64_t)1, 1,
                       1, 1, 1, s_hat);
    return ensei::launch_status();
}

int ensei_bfv_encrypt(ensei_bfv_ctx *ctx, const uint32_t *x_hat, int64_t B, int C, int64_t F, const uint32_t *s_hat,
                      const int32_t *e, uint64_t seed_a, uint64_t ct_index0, uint32_t *ct, void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!x_hat || !s_hat || !e || !ct || B <= 0) return ENSEI_ERR_ARG;
    Geometry gm;
    if (!geometry(ctx->K.n, C, F, &gm)) return ENSEI_ERR_SHAPE;
    if (F > ctx->K.n && F % ctx->K.n) return ENSEI_ERR_SHAPE;
    if (!aligned4(x_hat) || !aligned4(s_hat) || !aligned4(e) || !aligned4(ct)) return ENSEI_ERR_ALIGN;
    const int64_t count = B * gm.G * gm.KC, n = ctx->K.n;
    if (count > 0x7fffffff) return ENSEI_ERR_LIMIT;
    const size_t ctb = (size_t)count * 4 * n * 4;
    if (ensei::overlaps(ct, ctb, x_hat, (size_t)B * C * F * 4) || ensei::overlaps(ct, ctb, s_hat, (size_t)4 * n * 4) ||
        ensei::overlaps(ct, ctb, e, (size_t)count * n * 4))
        return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(bfv_encrypt_kernel, dim3((unsigned)count), dim3(kNT), lds_bytes(ctx, 2), (hipStream_t)stream, ctx->K, x_hat, C,
                       F, gm.P, gm.Fp, gm.G, gm.KC, s_hat, e, seed_a, ct_index0, ct);
    return ensei::launch_status();
}

int ensei_bfv_encode_filters(ensei_bfv_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F,
                             uint32_t *w_enc, void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!w_hat || !w_enc || Cout <= 0) return ENSEI_ERR_ARG;
    Geometry gm;
    if (!geometry(ctx->K.n, Cin, F, &gm)) return ENSEI_ERR_SHAPE;
    if (!aligned4(w_hat) || !aligned4(w_enc)) return ENSEI_ERR_ALIGN;
    const int64_t count = (int64_t)Cout * gm.G * gm.KC, n = ctx->K.n;
    if (count > 0x7fffffff) return ENSEI_ERR_LIMIT;
    if (ensei::overlaps(w_enc, (size_t)count * 4 * n * 4, w_hat, (size_t)Cout * Cin * F * 4)) return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(bfv_encode_kernel<0>, dim3((unsigned)count), dim3(kNT), lds_bytes(ctx, 2), (hipStream_t)stream, ctx->K, w_hat,
                       Cin, F, gm.P, gm.Fp, gm.G, gm.KC, w_enc);
    return ensei::launch_status();
}

int ensei_bfv_encode_masks(ensei_bfv_ctx *ctx, const uint32_t *r, int64_t count, uint32_t *mask_enc, void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!r || !mask_enc || count <= 0) return ENSEI_ERR_ARG;
    if (count > 0x7fffffff) return ENSEI_ERR_LIMIT;
    if (!aligned4(r) || !aligned4(mask_enc)) return ENSEI_ERR_ALIGN;
    const int64_t n = ctx->K.n;
    if (ensei::overlaps(mask_enc, (size_t)count * 2 * n * 4, r, (size_t)count * n * 4)) return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(bfv_encode_kernel<1>, dim3((unsigned)count), dim3(kNT), lds_bytes(ctx, 2), (hipStream_t)stream, ctx->K, r, 1,
                       (int64_t)1, 1, 1, 1, 1, mask_enc);
    return ensei::launch_status();
}

int ensei_bfv_homconv(ensei_bfv_ctx *ctx, const uint32_t *ct_in, const uint32_t *w_enc, const uint32_t *mask_enc,
                      int64_t B, int Cin, int Cout, int64_t F, uint32_t *ct_out, void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!ct_in || !w_enc || !mask_enc || !ct_out || B <= 0 || Cout <= 0) return ENSEI_ERR_ARG;
    Geometry gm;
    if (!geometry(ctx->K.n, Cin, F, &gm)) return ENSEI_ERR_SHAPE;
    if (!aligned4(ct_in) || !aligned4(w_enc) || !aligned4(mask_enc) || !aligned4(ct_out)) return ENSEI_ERR_ALIGN;
    const int64_t n = ctx->K.n, nout = B * Cout * gm.KC;
    const size_t outb = (size_t)nout * 4 * n * 4;
    if (ensei::overlaps(ct_out, outb, ct_in, (size_t)B * gm.G * gm.KC * 4 * n * 4) ||
        ensei::overlaps(ct_out, outb, w_enc, (size_t)Cout * gm.G * gm.KC * 4 * n * 4) ||
        ensei::overlaps(ct_out, outb, mask_enc, (size_t)nout * 2 * n * 4))
        return ENSEI_ERR_OVERLAP;
    const int64_t blocks = ((n + kNT - 1) / kNT) * 2 * gm.KC * ((Cout + kOB - 1) / kOB) * ((B + kBB - 1) / kBB);
    if (blocks > 0x7fffffff) return ENSEI_ERR_LIMIT;
    hipLaunchKernelGGL(bfv_homconv_kernel, dim3((unsigned)blocks), dim3(kNT), 0, (hipStream_t)stream, ctx->K, ct_in,
                       w_enc, mask_enc, B, gm.G, Cout, gm.KC, ct_out);
    return ensei::launch_status();
}

int ensei_bfv_decrypt(ensei_bfv_ctx *ctx, const uint32_t *ct, const uint32_t *s_hat, int64_t count, uint32_t *v,
                      void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!ct || !s_hat || !v || count <= 0) return ENSEI_ERR_ARG;
    if (count > 0x7fffffff) return ENSEI_ERR_LIMIT;
    if (!aligned4(ct) || !aligned4(s_hat) || !aligned4(v)) return ENSEI_ERR_ALIGN;
    const int64_t n = ctx->K.n;
    if (ensei::overlaps(v, (size_t)count * n * 4, ct, (size_t)count * 4 * n * 4) ||
        ensei::overlaps(v, (size_t)count * n * 4, s_hat, (size_t)4 * n * 4))
        return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(bfv_decrypt_kernel, dim3((unsigned)count), dim3(kNT), lds_bytes(ctx, 1), (hipStream_t)stream, ctx->K, ct, s_hat,
                       v);
    return ensei::launch_status();
}

int ensei_bfv_rerandomize(ensei_bfv_ctx *ctx, uint32_t *ct, int64_t count, const uint32_t *pk, uint64_t seed_r,
                          uint64_t ct_index0, uint32_t flood, void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!ct || !pk || count <= 0 || flood >= 0x80000000u) return ENSEI_ERR_ARG;
    if (count > 0x7fffffff) return ENSEI_ERR_LIMIT;
    if (!aligned4(ct) || !aligned4(pk)) return ENSEI_ERR_ALIGN;
    const int64_t n = ctx->K.n;
    if (ensei::overlaps(ct, (size_t)count * 4 * n * 4, pk, (size_t)4 * n * 4)) return ENSEI_ERR_OVERLAP;
    hipLaunchKernelGGL(bfv_rerandomize_kernel, dim3((unsigned)count), dim3(kNT), lds_bytes(ctx, 3), (hipStream_t)stream, ctx->K, ct, pk,
                       seed_r, ct_index0, flood);
    return ensei::launch_status();
}

int ensei_bfv_fold(ensei_bfv_ctx *ctx, const uint32_t *v, int64_t B, int C, int64_t F, int negate, uint32_t *y,
                   void *stream) {
    int st = check_bfv(ctx);
    if (st) return st;
    if (!v || !y || B <= 0 || (negate != 0 && negate != 1)) return ENSEI_ERR_ARG;
    Geometry gm;
    if (!geometry(ctx->K.n, 1, F, &gm)) return ENSEI_ERR_SHAPE;
    if (C <= 0) return ENSEI_ERR_ARG;
    if (!aligned4(v) || !aligned4(y)) return ENSEI_ERR_ALIGN;
    const int64_t total = B * C * F, n = ctx->K.n;
    if (ensei::overlaps(y, (size_t)total * 4, v, (size_t)B * C * gm.KC * n * 4)) return ENSEI_ERR_OVERLAP;
    if ((total + 255) / 256 > 0x7fffffff) return ENSEI_ERR_LIMIT;
    hipLaunchKernelGGL(bfv_fold_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, v, B,
                       C, F, (int)n, gm.P, gm.Fp, gm.KC, ctx->K.t, ctx->K.one_sh[0], negate, y);
    return ensei::launch_status();
}

}  // extern "C"
