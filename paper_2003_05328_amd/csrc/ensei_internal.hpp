// Internal declarations shared by the HIP sources of libensei.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/ensei.h"

struct ensei_ctx {
    int device;
    uint32_t p;         // prime modulus, 3 <= p < 2^22
    uint32_t g;         // smallest primitive root of p
    uint64_t delta;     // floor(2^64 / p)
    int max_log;        // largest log2(L) with L | p-1, capped at 7
    int num_cus;        // compute units of the device (persistent-kernel grids)
    // Device twiddle tables: for direction d (0 forward, 1 inverse) and each
    // length L = 2^l (1 <= l <= 7), L/2 entries (omega_L^j, floor(omega_L^j 2^24 / p))
    // starting at entry d * 127 + (L/2 - 1).
    uint2 *d_tw;
    // Thresholds of the rounded-Gaussian error sampler (ensei_sample_errors),
    // on the host and on the device: floor(2^48 P(|e| <= k)), k < 32.
    uint64_t cdt[32];
    uint64_t *d_cdt;
};

namespace ensei {

constexpr int kTwPerDir = 127;
// Launch facts computed once per device and kernel (occupancy, a raised
// dynamic-LDS limit) are cached in atomics indexed by device; devices past
// this count are not cached.
constexpr int kMaxDevices = 64;
constexpr int kCdtSize = 32, kCdtBits = 48;  // error sampler: thresholds, and their grid 2^-48

// Host-side checks shared by the entry points.
int check_ctx(const ensei_ctx *ctx);
bool overlaps(const void *a, size_t an, const void *b, size_t bn);
int launch_status();
int ilog2_pow2(int v);  // log2(v) if v is a power of two >= 2, else -1

// ------------------------------------------------------- Z_p on the VALU --
// Residues live in [0, 2p) between butterfly stages ("lazy" reduction);
// p < 2^22 keeps every operand of a 24-bit multiply below 2^24.

// Low 32 bits of a 24 x 24-bit product (v_mul_u32_u24, full rate).
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return (a & 0xffffffu) * (b & 0xffffffu); }

// The same product, kept as one instruction: without the asm the compiler
// may reassociate q1*p + q2*p into (q1+q2)*p, whose operand no longer fits
// 24 bits, and fall back to the quarter-rate 32-bit multiply.
__device__ __forceinline__ uint32_t mul24_pinned(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// a * w mod p, lazily reduced to [0, 2p), for a < 2^24, w < p and
// wq = floor(w * 2^24 / p) (Shoup's precomputed quotient with a 2^24 scale).
// q = floor(a * wq / 2^24) is floor(a w / p) or one less, so
// a w - q p lies in [0, 2p) and is exact modulo 2^32. Six full-rate ops.
__device__ __forceinline__ uint32_t mulmod_lazy(uint32_t a, uint32_t w, uint32_t wq, uint32_t p) {
    uint64_t prod = (uint64_t)(a & 0xffffffu) * (wq & 0xffffffu);
    uint32_t q = (uint32_t)(prod >> 24);
    return mul24(a, w) - mul24_pinned(q, p);
}

// mulmod_lazy for a twiddle in scalar registers (w, wq wave-uniform), every
// multiply pinned to the full-rate 24-bit instructions: where the compiler
// cannot bound a below 2^24 it would otherwise keep the masks and fall back
// to the quarter-rate 32-bit multiply.
__device__ __forceinline__ uint32_t mulmod_lazy_su(uint32_t a, uint32_t w, uint32_t wq, uint32_t p) {
    uint32_t lo, hi, aw, qp;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(lo) : "s"(wq), "v"(a));
    asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(hi) : "s"(wq), "v"(a));
    const uint32_t q = __builtin_amdgcn_alignbit(hi, lo, 24);
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(aw) : "s"(w), "v"(a));
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(qp) : "s"(p), "v"(q));
    return aw - qp;
}

// x mod p up to one p, for x < 2^24 and 256 < p: with m = floor(2^32 / p),
// q = floor(x m / 2^32) is floor(x / p) or one less, so x - q p lies in
// [0, 2p). Three full-rate ops.
__device__ __forceinline__ uint32_t reduce_2p(uint32_t x, uint32_t m, uint32_t p) {
    uint32_t q, qp;
    asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(q) : "s"(m), "v"(x));
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(qp) : "s"(p), "v"(q));
    return x - qp;
}

// x in [0, 2m) -> [0, m): unsigned min picks x when x < m (x - m wraps high).
__device__ __forceinline__ uint32_t reduce_once(uint32_t x, uint32_t m) {
    uint32_t y = x - m;
    return y < x ? y : x;  // y < x exactly when x >= m
}

// --------------------------------------------------- a-word generator --
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014): output number k
// of the generator seeded with x is mix(x + k * gamma). Word j < n of
// ciphertext q (q = (b F + f) C + c, counted from ct_index0) is output number
// (ct_index0 + q) n + j + 1 of the generator seeded with seed_a.
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------ HomConv --
// One HomConv problem of a launch; a multi-problem launch reads an array of
// these from device memory. tile0 is the problem's first tile in the
// launch's concatenated tile space (tiles of 64 rows x 64 words per (b, f)).
// Seeded input (ensei_homconv_seeded): ct_in is unused; the b words are
// b_in [B][F][Cin] and the a-words come from (seed_a, idx0).
struct HcLayer {
    const uint64_t *ct_in;
    const int8_t *w_pack;
    const uint32_t *r;
    uint64_t *ct_out;
    int64_t F, B, tile0, n_tiles;
    int Cin, Cout, n, n_ot, n_jt, n_ks, n_items, pad;
    const uint64_t *b_in;
    uint64_t seed_a, idx0;
};

// Tile schedule of a HomConv launch: persistent workgroups, and chunk = 0
// (one contiguous tile range per workgroup) or the size of the chunks dealt
// out round-robin.
struct HcSchedule {
    int blocks;
    int64_t chunk;
};

constexpr int kPairedCin = 48;  // ensei_homconv's paired limb scheme from this many input channels on
// Inputs this narrow run on their own barrier-free kernel (folded fragments),
// launched as a single problem; batched launches keep them out of the
// multi-problem table.
constexpr int kNarrowCin = 8;

// 16-byte weight-fragment items per (f, K step, row tile) unit of each scheme
inline int frag_items(int Cin, bool paired) { return paired ? 768 : 256 * ((Cin + 15) / 16); }
size_t wpack_bytes_as(int Cout, int Cin, int64_t F, bool paired);
int pack_weights_as(const ensei_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F, bool paired,
                    int8_t *w_pack, hipStream_t stream);
// HomConv's size limits alone (ENSEI_ERR_ARG / ENSEI_ERR_LIMIT).
int homconv_sizes(int64_t batch, int Cin, int Cout, int64_t F, int n);
// Checks one problem's sizes and fills its derived fields (tile0 = 0).
// seeded: ct_in points at the b words [B][F][Cin] of seeded ciphertexts
// (the caller sets seed_a and idx0)
int homconv_problem(const ensei_ctx *ctx, HcLayer *P, const uint64_t *ct_in, const int8_t *w_pack, const uint32_t *r,
                    int64_t B, int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, size_t wbytes,
                    bool seeded = false);
// Whether a single problem (paired fragments) runs on the deep-layer kernel;
// batched launches keep such layers out of the multi-problem table.
bool homconv_deep_fits(const HcLayer &P, bool seeded = false);
// Launches the matrix-core HomConv over problems[0..nlayers) (host copies;
// dev_table holds the same array in device memory when nlayers > 1).
// seeded: the problems' inputs are seeded (b_in, seed_a, idx0)
int homconv_launch(const ensei_ctx *ctx, const HcLayer *problems, const HcLayer *dev_table, int nlayers, bool paired,
                   HcSchedule sched, hipStream_t stream, bool seeded = false);

}  // namespace ensei
