// HomConv: for every (image b, frequency f) an exact integer contraction
//   ct_out(b, :, f) = W^_f (Cout x Cin) . ct_in(b, :, f) (Cin x (n+1))  mod 2^64
// plus Delta * r[b][o][f] on the b word (HomShare). Ciphertexts are stored
// word-major, ct[b][f][j][c]: for one (b, f) the block is a (n+1) x C matrix
// whose row j holds word j of all C channels.
//
// Matrix-core kernel (ensei_homconv). Both operands are split into signed
// bytes so the i8 MFMA (v_mfma_i32_16x16x64_i8) does the multiplies:
//   - a ciphertext word c is written in balanced base 256,
//     c = sum_{k<8} d_k 256^k mod 2^64 with d_k in [-128, 127]; the digits are
//     the bytes of c + 0x8080...80, each xor 0x80 (the carry out of the top
//     digit vanishes mod 2^64);
//   - W^ < 2^22 as w0 + 256 w1 + 65536 w2, the same balanced digits
//     (ensei_pack_weights).
//   Then sum_i W^ c = sum_{s<8} 256^s acc_s mod 2^64 with
//   acc_s = sum_i sum_{l<=2, l<=s} w_l[i] d_{s-l}[i], an exact i32 sum
//   (|acc_s| <= 3 * Cin * 2^14 < 2^31 for Cin <= 32768). Products with
//   l + k >= 8 are multiples of 2^64 and are never formed.
//   The kernel's two K layouts (limbs folded into K, or one limb pair per
//   instruction) are described at the kernel.
//
// Three kernels share these operand layouts; ensei_homconv picks one per
// layer (homconv_launch):
//   - homconv_mfma_kernel, the streaming kernel (every layer, and every
//     layer of a multi-problem launch): a tile is (b, f, 64 rows o, 64
//     columns j) and a unit a (tile, 64-channel K step). With C = 64 channels
//     both the unit's input words and the tile's output words are one
//     contiguous 32 KB block, which is what lets the kernel stream at HBM
//     rate. One 8-wave workgroup per CU walks a contiguous range of tiles (row
//     tiles fastest, so extra row tiles of a (b, f, columns) reuse its input
//     from L2), two units ahead: the next two units' words, weight fragments
//     and masks are in flight while the current unit is converted to digit
//     planes and contracted on the MFMAs. Each wave owns 16 columns x 32 rows
//     and the eight shift accumulators in registers;
//   - homconv_narrow_kernel (Cin <= 8): barrier-free waves for the
//     write-bound narrow-input layers;
//   - homconv_deep_kernel (several row tiles, Cin <= 256): the input of a
//     32-column block converted once into LDS for all of its row tiles.
// In all of them the rows of the MFMA's A operand are permuted so that every
// lane ends up with 8 consecutive output rows of one column: after the
// recombination each lane stores whole 64-byte runs of ct_out straight from
// its registers.
#include <type_traits>

#include "ensei_internal.hpp"

namespace ensei {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kPlaneBytes = 64 * 4 * 16;  // one digit plane: 64 columns x 4 channel groups x 16 bytes
constexpr uint32_t kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
// Cache policy of a streaming store: non-temporal (the line is not kept in
// the caches for reuse). A write stream issued this way no longer delays the
// reads that the same waves interleave with it.
constexpr int kStoreStream = 2;

// Raw buffer descriptor over [base, base + nbytes): accesses at or past nbytes
// read zero / are dropped by the hardware range check.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)nbytes, kRsrcWord3);
}

// Channel group sc of column col lives in slot sc ^ ((col >> 1) & 3) of the
// column's four 16-byte slots: both the 8-byte writes (lanes over 2 columns x
// 4 groups x 2 halves) and the MFMA's 16-byte reads (lanes over 16 columns)
// then touch distinct banks.
__device__ __forceinline__ int plane_slot(int col, int sc) { return col * 4 + (sc ^ ((col >> 1) & 3)); }

// A pointer every lane of the wave holds, moved to scalar registers so that
// address arithmetic on it stays on the scalar unit.
__device__ __forceinline__ const uint8_t *uniform_ptr(const uint8_t *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const uint8_t *>(((uint64_t)hi << 32) | lo);
}

// Global-memory load from a wave-uniform base plus a 32-bit lane offset (the
// scalar-base addressing form of the load instructions).
template <typename T>
__device__ __forceinline__ T load_global(const uint8_t *base, uint32_t off) {
    using gptr = __attribute__((address_space(1))) const T *;
    return *(gptr)(uintptr_t)(base + off);
}

// 4 x 4 byte transpose: y_k byte i = x_i byte k.
__device__ __forceinline__ void transpose4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t &y0,
                                           uint32_t &y1, uint32_t &y2, uint32_t &y3) {
    const uint32_t t0 = __builtin_amdgcn_perm(x1, x0, 0x05010400u);  // x0b0 x1b0 x0b1 x1b1
    const uint32_t t1 = __builtin_amdgcn_perm(x1, x0, 0x07030602u);  // x0b2 x1b2 x0b3 x1b3
    const uint32_t t2 = __builtin_amdgcn_perm(x3, x2, 0x05010400u);  // x2b0 x3b0 x2b1 x3b1
    const uint32_t t3 = __builtin_amdgcn_perm(x3, x2, 0x07030602u);  // x2b2 x3b2 x2b3 x3b3
    y0 = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    y1 = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    y2 = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    y3 = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Stores the 8 words res[rb][i] a lane holds after the contraction: rows
// row0 + 8 g + 4 rb + i of output column col (g = lane / 16), into the block
// rs addresses as [column][Cout]. Rows at or past Cout are not written.
// WIDE_STORE (Cout even): 16-byte chunk c of lane row g (lanes 16 g + l16) is
// X[c]; a 4 x 4 transpose across the lane rows (swap halves, then odd/even
// rows) leaves X[q] = rows 8 q + 2 g, 8 q + 2 g + 1, so the four lane rows of
// one column hold 64 contiguous bytes in each X[q], and store q writes them.
// FULL_LINES: neighbouring lanes (the columns 2 p, 2 p + 1) first trade one
// chunk per pair (X[2 m], X[2 m + 1]):
// afterwards the even lane holds rows 16 m .. 16 m + 7 and the odd lane rows
// 16 m + 8 .. 16 m + 15 of column 2 p for one store, and of column 2 p + 1
// for the next, so every store instruction writes whole 128-byte lines
// (half-line stores interleaved with a wave's own loads stream markedly
// slower; where a kernel is not store-bound the exchange costs more than it
// gains). col's parity must be the lane's. shuffle = false skips the
// exchanges (for stores that the range check drops anyway). CPOL is the
// stores' cache policy (kStoreStream: non-temporal).
template <bool WIDE_STORE, bool FULL_LINES, int CPOL>
__device__ __forceinline__ void store_lane_words(const uint64_t (&res)[2][4], __amdgpu_buffer_rsrc_t rs, int col,
                                                 int row0, int g, int Cout, bool shuffle) {
    const uint32_t col_off = (uint32_t)(col * Cout * 8);
    if (WIDE_STORE) {
        uint32_t X[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint64_t w0 = res[c >> 1][2 * (c & 1)], w1 = res[c >> 1][2 * (c & 1) + 1];
            X[c][0] = (uint32_t)w0;
            X[c][1] = (uint32_t)(w0 >> 32);
            X[c][2] = (uint32_t)w1;
            X[c][3] = (uint32_t)(w1 >> 32);
        }
        if (shuffle) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const auto t = __builtin_amdgcn_permlane32_swap(X[c][d], X[c + 2][d], false, false);
                    X[c][d] = t[0];
                    X[c + 2][d] = t[1];
                }
#pragma unroll
                for (int c = 0; c < 4; c += 2) {
                    const auto t = __builtin_amdgcn_permlane16_swap(X[c][d], X[c + 1][d], false, false);
                    X[c][d] = t[0];
                    X[c + 1][d] = t[1];
                }
            }
        }
        if (!FULL_LINES) {
            const int o = row0 + 2 * g;  // + 8 q: rows of store q
            const uint32_t off = col_off + (uint32_t)(o * 8);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const u32x4 d = {X[q][0], X[q][1], X[q][2], X[q][3]};
                __builtin_amdgcn_raw_buffer_store_b128(d, rs, (int)(o + 8 * q < Cout ? off + 64 * q : 0x80000000u), 0,
                                                       CPOL);
            }
            return;
        }
        const bool odd = col & 1;
        if (shuffle) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    // even lane sends X[2m + 1] and receives the odd lane's X[2m]
                    const uint32_t send = odd ? X[2 * m][d] : X[2 * m + 1][d];
                    const uint32_t recv = (uint32_t)__builtin_amdgcn_mov_dpp((int)send, 0xB1, 0xF, 0xF, false);
                    if (odd)
                        X[2 * m][d] = recv;
                    else
                        X[2 * m + 1][d] = recv;
                }
        }
        // store 2 m + h: column (col & ~1) + h, rows 16 m + 8 (col & 1) + 2 g, + 1
        const int o = row0 + 8 * (int)odd + 2 * g;
        const uint32_t pair_off = (uint32_t)((col & ~1) * Cout * 8) + (uint32_t)(o * 8);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // X[2m + h] holds column (col & ~1) + h in both lanes of the pair
                const int q = 2 * m + h;
                const u32x4 d = {X[q][0], X[q][1], X[q][2], X[q][3]};
                __builtin_amdgcn_raw_buffer_store_b128(
                    d, rs,
                    (int)(o + 16 * m < Cout ? pair_off + (uint32_t)(h * Cout * 8) + 128u * m : 0x80000000u), 0, CPOL);
            }
    } else {
        const int o = row0 + 8 * g;
        const uint32_t off = col_off + (uint32_t)(o * 8);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint64_t w = res[q >> 2][q & 3];
            const u32x2 d = {(unsigned)w, (unsigned)(w >> 32)};
            __builtin_amdgcn_raw_buffer_store_b64(d, rs, (int)(o + q < Cout ? off + 8 * q : 0x80000000u), 0, CPOL);
        }
    }
}

// Position of one work unit: layer L, global tile t, and within the layer's
// tile the row tile ot, column tile jt, K step ks, frequency f and image b.
struct HcCoord {
    int L, ot, jt, ks;
    int64_t t, f, b;
};

// Data of one unit in flight: 8 words per thread, 2 weight-fragment items, 1 mask.
// afresh: the weight fragments were loaded for this unit; otherwise the
// LDS buffer of this parity already holds them (akey: their address).
struct HcBuf {
    u32x4 w[4];
    v4i a[2];
    uint32_t r;
    uint64_t akey;
    bool afresh;
};

constexpr int kHcThreads = 512;

// Shift accumulators -> one u64 word, mod 2^64:
//   sum_{s<4} 256^s acc_s exactly (signed), plus 2^32 (sum_{s>=4} 256^(s-4) acc_s mod 2^32).
// SMALL: Cin <= kSmallCin, so acc_0 + 256 acc_1 and acc_2 + 256 acc_3 are exact i32
// values (|acc_s| <= 3 Cin 2^14) and the low part needs one 64-bit add.
constexpr int kSmallCin = 169;

template <bool SMALL>
__device__ __forceinline__ uint64_t recombine(int a0, int a1, int a2, int a3, int a4, int a5, int a6, int a7) {
    uint64_t lo;
    if (SMALL) {
        const int32_t u = (int32_t)((uint32_t)a0 + ((uint32_t)a1 << 8));
        const int32_t v = (int32_t)((uint32_t)a2 + ((uint32_t)a3 << 8));
        lo = (uint64_t)(int64_t)u + ((uint64_t)(int64_t)v << 16);
    } else {
        lo = (uint64_t)(int64_t)a0 + ((uint64_t)(int64_t)a1 << 8) + ((uint64_t)(int64_t)a2 << 16) +
             ((uint64_t)(int64_t)a3 << 24);
    }
    const uint32_t h = (uint32_t)a4 + ((uint32_t)a5 << 8) + ((uint32_t)a6 << 16) + ((uint32_t)a7 << 24);
    return lo + ((uint64_t)h << 32);
}

// PAIRED = false ("folded" limbs): one MFMA's 64-long K holds 16 channels x
// 4 limb slots (slot l < 3 pairs weight limb l with digit plane s - l, slot 3
// meets a zero plane), one instruction per shift s and 16 channels: 32 MFMAs
// per 64 channels and row block. Best when Cin is small.
// PAIRED = true: K holds 64 channels of one weight limb l and one digit
// plane k, one instruction per pair (l, k) with l + k < 8 accumulating into
// shift l + k: 21 MFMAs per 64 channels and row block and a quarter of the
// LDS operand reads. Used when Cin >= 48.
// WIDE_STORE: Cout is even, so the two words of every 16-byte store are
// both inside the output row or both outside it.
// MULTI: the launch walks the concatenated tiles of several HomConv
// problems (layers of uneven shapes) read from a device table; otherwise the
// one problem comes in the kernel arguments.
// SEEDED: the input ciphertexts are seeded (ensei_homconv_seeded): words
// j < n are generated from the public stream where they would be loaded,
// and only the b words (column n) are read, from b_in.
// Tile schedule: with chunk == 0 each workgroup takes one contiguous range of
// tiles; otherwise tiles are dealt out in chunks of `chunk` consecutive tiles,
// chunk c to workgroup c mod gridDim.x.
template <bool PAIRED, bool WIDE_STORE, bool MULTI, bool SEEDED>
__global__ __launch_bounds__(kHcThreads) void homconv_mfma_kernel(HcLayer one, const HcLayer *__restrict__ table,
                                                                  int nlayers, int64_t total_tiles, int64_t chunk,
                                                                  uint64_t delta) {
    constexpr int kAItems = PAIRED ? 3 * 4 * 64 : 4 * 4 * 64;  // [limb 3 | sc 4][row block 4][lane 64] x 16 B
    constexpr int kA = kAItems * 16;
    constexpr int kZeroPlanes = PAIRED ? 0 : 2;  // the folded scheme reads planes -2, -1 as zero
    // Two LDS buffers, for units of even and odd index, each holding digit
    // planes k = -kZeroPlanes..7, the unit's weight fragments and its 64 masks.
    // A unit's operands are written while other waves may still be reading
    // the previous unit's, so one barrier per unit is enough.
    constexpr int kLdsBuf = (8 + kZeroPlanes) * kPlaneBytes + kA + 64 * 4;
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kLdsBuf];
    auto planes = [&](int lb) { return lds + lb * kLdsBuf + kZeroPlanes * kPlaneBytes; };  // plane k at + k * kPlaneBytes
    auto lds_a = [&](int lb) { return lds + lb * kLdsBuf + (8 + kZeroPlanes) * kPlaneBytes; };
    auto lds_r = [&](int lb) { return reinterpret_cast<uint32_t *>(lds + lb * kLdsBuf + (8 + kZeroPlanes) * kPlaneBytes + kA); };

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, l16 = lane & 15;
    const int cg = wave & 3, rg = wave >> 2;  // MFMA role: columns 16 cg.., rows 32 rg..
    // problem L's parameters (wave-uniform: scalar loads from the table)
    auto layer = [&](int L) -> HcLayer { return MULTI ? table[L] : one; };

    // this block's tiles: [t_lo, t_hi) when contiguous; else its chunks
    const int64_t G = gridDim.x;
    int64_t t_lo = 0, t_hi = 0;
    if (chunk == 0) {
        const int64_t per = total_tiles / G, extra = total_tiles % G;
        t_lo = blockIdx.x * per + (blockIdx.x < extra ? blockIdx.x : extra);
        t_hi = t_lo + per + (blockIdx.x < extra ? 1 : 0);
    }
    // number of this block's tiles below x
    auto owned_below = [&](int64_t x) -> int64_t {
        if (chunk == 0) return (x < t_lo ? t_lo : x > t_hi ? t_hi : x) - t_lo;
        const int64_t S = G * chunk, rem = x % S - (int64_t)blockIdx.x * chunk;
        return x / S * chunk + (rem < 0 ? 0 : rem > chunk ? chunk : rem);
    };
    // units = sum over problems of (owned tiles) x (K steps)
    int64_t n_units = 0;
    for (int L = 0; L < nlayers; ++L) {
        const HcLayer P = layer(L);
        n_units += (owned_below(P.tile0 + P.n_tiles) - owned_below(P.tile0)) * P.n_ks;
    }
    if (n_units == 0) return;

    if (kZeroPlanes > 0) {
        constexpr int kZero16 = (kZeroPlanes > 0 ? kZeroPlanes : 1) * kPlaneBytes / 16;  // per buffer
        for (int i = tid; i < 2 * kZero16; i += kHcThreads)
            reinterpret_cast<uint4 *>(lds + (i / kZero16) * kLdsBuf)[i % kZero16] = make_uint4(0, 0, 0, 0);
    }

    // load role: column ld_col, channel group ld_sc, half ld_h (8 channels)
    const int ld_col = tid >> 3, ld_sc = (tid >> 1) & 3, ld_h = tid & 1;
    const int b_col = cg * 16 + l16;  // this lane's B column
    // folded: plane s - g (slot 3: the zero plane); paired: plane k, channel group g
    const int b_base = PAIRED ? plane_slot(b_col, g) * 16 : (g == 3 ? -1 : -g) * kPlaneBytes;
    const int b_step = PAIRED ? kPlaneBytes : (g == 3 ? 0 : kPlaneBytes);
    const int out_row = 32 * rg + 8 * g;  // first of this lane's 8 output rows in the tile

    auto issue = [&](const HcCoord &u, HcBuf &buf) {
        const HcLayer P = layer(u.L);
        const int Cin = P.Cin, Cout = P.Cout;
        const int64_t F = P.F, rowlen = (int64_t)P.n + 1;
        const int col = u.jt * 64 + ld_col;
        // columns past n read zero; an 8-channel group that starts past Cin
        // is not read at all (no traffic), one that straddles it reads the next
        // column's words, which meet zero weights
        const bool any = ld_sc * 16 + ld_h * 8 < Cin - u.ks * 64;
        if (SEEDED) {
            // column n: the b words of the 8 channels from b_in [B][F][Cin]
            // (outside the column tile holding it nothing is read); the words
            // of columns below n are generated when the unit is converted
            const int c0 = u.ks * 64 + ld_sc * 16 + ld_h * 8;
            const uint8_t *bblk = uniform_ptr(reinterpret_cast<const uint8_t *>(P.b_in + (u.b * F + u.f) * Cin));
            const __amdgpu_buffer_rsrc_t rb = make_rsrc(bblk, u.jt == P.n_jt - 1 ? (uint32_t)(Cin * 8) : 0u);
            const uint32_t boff = any && col == P.n ? (uint32_t)(c0 * 8) : 0x80000000u;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                buf.w[q] = __builtin_amdgcn_raw_buffer_load_b128(rb, (int)(boff + 16 * q), 0, 0);
        } else {
            const uint8_t *blk =
                uniform_ptr(reinterpret_cast<const uint8_t *>(P.ct_in + (u.b * F + u.f) * rowlen * Cin));
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(blk, (uint32_t)(rowlen * Cin * 8));
            const uint32_t off =
                any ? (uint32_t)(((int64_t)col * Cin + u.ks * 64 + ld_sc * 16 + ld_h * 8) * 8) : 0x80000000u;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                buf.w[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16 * q), 0, 0);
        }
        // the unit's weight fragments: n_items contiguous 16-byte items, item k
        // read by thread k % 512 (items past n_items read zero, with no traffic)
        // Consecutive units mostly share them (same problem, f, K step and row
        // tile for every column tile): when the unit two back, whose LDS buffer
        // this unit reuses, had the same ones, nothing is read or rewritten.
        const int64_t unit = ((int64_t)u.f * P.n_ks + u.ks) * P.n_ot + u.ot;
        const uint8_t *abase = uniform_ptr(reinterpret_cast<const uint8_t *>(P.w_pack) + unit * P.n_items * 16);
        buf.afresh = (uint64_t)abase != buf.akey;
        buf.akey = (uint64_t)abase;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(abase, buf.afresh ? (uint32_t)(P.n_items * 16) : 0u);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(ra, (tid + kHcThreads * j) * 16, 0, 0);
            buf.a[j] = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
        }
        // masks are needed only in the column tile holding the b word (j = n),
        // and only by the first wave: every other load is out of range and
        // generates no memory traffic
        const int o = u.ot * 64 + tid;
        const __amdgpu_buffer_rsrc_t rr =
            make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(P.r + u.b * Cout * F + u.f)),
                      u.jt == P.n_jt - 1 ? (uint32_t)(((int64_t)(Cout - 1) * F + 1) * 4) : 0u);
        buf.r = __builtin_amdgcn_raw_buffer_load_b32(rr, (int)(tid < 64 && o < Cout ? (uint32_t)(o * F * 4) : 0x80000000u),
                                                     0, 0);
    };

    // coordinates of global tile t (K step 0); t past the end leaves c as is
    auto seek = [&](HcCoord &c, int64_t t) {
        if (t >= total_tiles) return;
        int L = 0;
        while (L + 1 < nlayers && t >= layer(L + 1).tile0) ++L;
        const HcLayer P = layer(L);
        int64_t x = t - P.tile0;
        c.L = L;
        c.t = t;
        c.ks = 0;
        c.ot = (int)(x % P.n_ot);
        x /= P.n_ot;
        c.jt = (int)(x % P.n_jt);
        x /= P.n_jt;
        c.f = x % P.F;
        c.b = x / P.F;
    };
    // the next unit in processing order: K steps, then row tiles, column
    // tiles, frequencies, images, problems; a new chunk is looked up
    auto advance = [&](HcCoord &c) {
        const HcLayer P = layer(c.L);
        if (++c.ks < P.n_ks) return;
        c.ks = 0;
        ++c.t;
        if (chunk != 0 && c.t % chunk == 0) {
            seek(c, c.t + (G - 1) * chunk);
            return;
        }
        if (++c.ot < P.n_ot) return;
        c.ot = 0;
        if (++c.jt < P.n_jt) return;
        c.jt = 0;
        if (++c.f < P.F) return;
        c.f = 0;
        if (++c.b < P.B) return;
        c.b = 0;
        if (c.L + 1 < nlayers) ++c.L;
    };
    // cur: the unit being contracted; cv: the next one, being converted;
    // nx: the last one issued
    HcCoord cur, cv, nx;
    seek(cur, chunk == 0 ? t_lo : (int64_t)blockIdx.x * chunk);
    v4i acc[8][2];

    // digit planes of one unit's 8 words per thread: 8 bytes of each plane,
    // in pl (u: the unit, whose position the seeded form needs to generate
    // its words)
    auto convert = [&](const HcCoord &u, const HcBuf &buf, uint32_t (&pl)[8][2]) {
        // seeded input: this thread's words j = col < n of its 8 channels,
        // from the public stream (zero where the words were loaded)
        uint64_t gen[8];
        if (SEEDED) {
            const HcLayer P = layer(u.L);
            const int col = u.jt * 64 + ld_col, c0 = u.ks * 64 + ld_sc * 16 + ld_h * 8;
            const bool on = c0 < P.Cin && col < P.n;
            const uint64_t q0 = P.idx0 + (uint64_t)((u.b * P.F + u.f) * P.Cin + c0);
            uint64_t z = P.seed_a + (q0 * (uint64_t)P.n + (uint64_t)col + 1) * kGamma;
            const uint64_t step = (uint64_t)P.n * kGamma;  // next channel, same word
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint64_t a = splitmix_mix(z);
                gen[i] = on ? a : 0ull;
                z += step;
            }
        }
        {
            uint32_t lo[8], hi[8];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint64_t v0 = (uint64_t)buf.w[q].y << 32 | buf.w[q].x;
                uint64_t v1 = (uint64_t)buf.w[q].w << 32 | buf.w[q].z;
                if (SEEDED) {  // a thread's words are either loaded or generated; the other part is zero
                    v0 += gen[2 * q];
                    v1 += gen[2 * q + 1];
                }
                v0 += 0x8080808080808080ull;
                v1 += 0x8080808080808080ull;
                lo[2 * q] = (uint32_t)v0;
                hi[2 * q] = (uint32_t)(v0 >> 32);
                lo[2 * q + 1] = (uint32_t)v1;
                hi[2 * q + 1] = (uint32_t)(v1 >> 32);
            }
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                transpose4(lo[4 * d], lo[4 * d + 1], lo[4 * d + 2], lo[4 * d + 3], pl[0][d], pl[1][d], pl[2][d],
                           pl[3][d]);
                transpose4(hi[4 * d], hi[4 * d + 1], hi[4 * d + 2], hi[4 * d + 3], pl[4][d], pl[5][d], pl[6][d],
                           pl[7][d]);
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            pl[k][0] ^= 0x80808080u;
            pl[k][1] ^= 0x80808080u;
        }
    };
    // a unit's digit planes, its weight fragments (when loaded for it) and its
    // masks into LDS buffer lb
    auto store_unit = [&](const uint32_t (&pl)[8][2], const HcBuf &buf, int lb) {
        const int pslot = plane_slot(ld_col, ld_sc) * 16 + ld_h * 8;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            *reinterpret_cast<u32x2 *>(planes(lb) + k * kPlaneBytes + pslot) = u32x2{pl[k][0], pl[k][1]};
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (buf.afresh && tid + kHcThreads * j < kAItems)
                reinterpret_cast<v4i *>(lds_a(lb))[tid + kHcThreads * j] = buf.a[j];
        if (tid < 64) lds_r(lb)[tid] = buf.r;
    };

    // MFMA phase of one unit; FRESH: the first product into each shift
    // accumulator starts from zero (the unit is the tile's first K step).
    // Interleaved (paired, words loaded), mid() runs in the same
    // straight-line code, so that its vector work (the next unit's
    // conversion) issues while the matrix cores run. The folded form (more
    // operand registers) and the seeded one (a generator whose long chains
    // leave the MFMAs bunched) convert before contracting instead.
    constexpr bool kInterleave = PAIRED && !SEEDED;
    auto contract = [&](auto fresh_tag, int lb, int sc_here, auto &&mid) {
        constexpr bool FRESH = decltype(fresh_tag)::value;
        const v4i zero = {0, 0, 0, 0};
        if (PAIRED) {
            v4i A[3][2];
#pragma unroll
            for (int l = 0; l < 3; ++l)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
                    A[l][rb] = reinterpret_cast<const v4i *>(lds_a(lb))[(l * 4 + rg * 2 + rb) * 64 + lane];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // (between instructions that differ with FRESH, so that it
                // is not moved out ahead of the caller's branch on it)
                if (kInterleave && k == 4) mid();
                const v4i B = *reinterpret_cast<const v4i *>(planes(lb) + b_base + k * b_step);
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    if (k + l >= 8) break;
                    // in this order shift k + l is first reached at k = 0 or l = 2
                    const bool first = FRESH && (k == 0 || l == 2);
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
                        acc[k + l][rb] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(A[l][rb], B, first ? zero : acc[k + l][rb], 0, 0, 0);
                }
            }
            // schedule: each MFMA followed by two of mid()'s vector instructions
            if (kInterleave) {
#pragma unroll
                for (int i = 0; i < 42; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
                }
            }
        } else {
#pragma unroll
            for (int sc = 0; sc < 4; ++sc) {
                if (sc >= sc_here) break;  // groups past Cin are zero
                v4i A[2];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
                    A[rb] = reinterpret_cast<const v4i *>(lds_a(lb))[(sc * 4 + rg * 2 + rb) * 64 + lane];
                const uint8_t *bp = planes(lb) + b_base + plane_slot(b_col, sc) * 16;
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const v4i B = *reinterpret_cast<const v4i *>(bp + s * b_step);
                    const bool first = FRESH && sc == 0;
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
                        acc[s][rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[rb], B, first ? zero : acc[s][rb], 0, 0, 0);
                }
            }
        }
    };

    // 8 output words of this lane: tile rows out_row + 4 rb + i of column b_col
    auto store_out = [&](const uint64_t (&res)[2][4], bool valid) {
        const HcLayer P = layer(cur.L);
        const int64_t F = P.F, rowlen = (int64_t)P.n + 1;
        const uint64_t *blk = P.ct_out + ((cur.b * F + cur.f) * rowlen + cur.jt * 64) * P.Cout;
        // columns past n fall outside the block and are dropped
        const uint32_t nbytes = valid ? (uint32_t)((rowlen - cur.jt * 64) * P.Cout * 8) : 0u;
        const __amdgpu_buffer_rsrc_t rs =
            make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(blk)), __builtin_amdgcn_readfirstlane(nbytes));
        store_lane_words<WIDE_STORE, false, 0>(res, rs, b_col, cur.ot * 64 + 32 * rg, g, P.Cout, valid);
    };

    // Two units' words in flight from the start; the entry issues the same
    // load and store sequence as every iteration (stores fully out of bounds)
    // so the waits see one static count on every incoming path. The first
    // unit is converted here; from then on each unit's conversion runs during
    // the previous unit's MFMAs.
    HcBuf buf0, buf1;
    buf0.akey = buf1.akey = 0;  // no fragments in either LDS buffer yet
    const uint64_t none[2][4] = {};
    nx = cur;
    issue(nx, buf0);
    store_out(none, false);
    if (n_units > 1) advance(nx);
    issue(nx, buf1);
    store_out(none, false);
    int64_t issued = n_units > 1 ? 2 : 1;
    cv = cur;
    {
        uint32_t pl[8][2];
        convert(cv, buf0, pl);
        store_unit(pl, buf0, 0);
    }
    advance(cv);
    __syncthreads();

    uint64_t res[2][4] = {};  // the last finished tile's words (kept across units)
    // one unit: its operands are in LDS buffer lb, its words were in bcur
    // (free again); the next unit's words are in bnxt and go to buffer lb ^ 1
    auto body = [&](HcBuf &bcur, HcBuf &bnxt, int lb) {
        const HcLayer P = layer(cur.L);
        const bool last_ks = cur.ks == P.n_ks - 1;

        // the unit two ahead reuses bcur (past the end: reissue the last
        // one, keeping the load count static)
        if (issued < n_units) {
            advance(nx);
            ++issued;
        }
        issue(nx, bcur);

        // this unit's MFMAs and the next unit's conversion (past the last
        // unit it converts words that are never read). Interleaved, the
        // conversion runs among the MFMAs and its LDS writes follow the
        // MFMAs' LDS reads; otherwise it comes first.
        uint32_t pl[8][2];
        auto conv = [&] { convert(cv, bnxt, pl); };
        if (!kInterleave) {
            conv();
            store_unit(pl, bnxt, lb ^ 1);
        }
        // 16-channel groups holding channels in this K step (folded scheme)
        const int sc_here = last_ks ? (P.Cin - 64 * (P.n_ks - 1) + 15) / 16 : 4;
        if (cur.ks == 0)
            contract(std::true_type{}, lb, sc_here, conv);
        else
            contract(std::false_type{}, lb, sc_here, conv);
        if (kInterleave) store_unit(pl, bnxt, lb ^ 1);

        // epilogue: recombine the shift accumulators (in every unit, so the
        // store count stays static; only the tile's last K step stores)
        auto recombine_all = [&](auto small_tag) {
            constexpr bool SMALL = decltype(small_tag)::value;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    res[rb][i] = recombine<SMALL>(acc[0][rb][i], acc[1][rb][i], acc[2][rb][i], acc[3][rb][i],
                                                  acc[4][rb][i], acc[5][rb][i], acc[6][rb][i], acc[7][rb][i]);
        };
        // only the tile's last K step recombines; the others issue the same
        // (dropped) stores so that the wait counts stay static
        if (last_ks) {
            if (P.Cin <= kSmallCin)
                recombine_all(std::true_type{});
            else
                recombine_all(std::false_type{});
            // HomShare: Delta * r on the b word (column n)
            if (cur.jt * 64 + 64 > P.n && cur.jt * 64 + b_col == P.n) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) res[rb][i] += delta * (uint64_t)lds_r(lb)[out_row + 4 * rb + i];
            }
        }
        store_out(res, last_ks);
        advance(cur);
        advance(cv);
        // buffer lb ^ 1 is complete and every wave is done with buffer lb
        __syncthreads();
    };

    for (int64_t it = 0; it < n_units / 2; ++it) {
        body(buf0, buf1, 0);
        body(buf1, buf0, 1);
    }
    if (n_units & 1) body(buf0, buf1, 0);
}

// Deep-layer HomConv (paired fragments, Cin <= 64 kDeepMaxKs, several
// 64-row output tiles): a block is (b, f, 32 columns j), and one 12-wave
// workgroup per CU walks a contiguous range of blocks. The block's words of
// every input channel are converted to digit planes in LDS once (up to 64 KB),
// then every (row-tile pair, K step) phase of the block contracts from there
// with no barrier in between: the conversion is shared by all Cout rows
// instead of being repeated per row tile. Eight compute waves hold 16 columns
// x 32 rows each, 128 rows (two row tiles) per phase. Four loader waves
// stream the coming blocks' words from HBM straight into a ring of LDS
// staging buffers (LDS-DMA buffer loads) while the compute waves contract the
// current one.
// The weight fragments come one of two ways:
//   - resident (AL): when the frequency's whole fragment set fits in LDS
//     beside the planes and the staging buffer (128 input channels, up to 256
//     outputs), the loader waves copy it there whenever a block of a new
//     frequency starts (a workgroup's blocks cover one or a few
//     frequencies), and the compute waves read it with the planes: they
//     issue no loads at all;
//   - streamed: each compute wave loads its own fragments from the L2 one
//     phase ahead (across block boundaries too) into two register sets used
//     in turn, so that no copy waits for a load in flight.
// The loader/compute split matters because a wave's memory counter retires
// in issue order: a compute wave that issued the HBM loads itself would, at
// its next wait for fragments, wait for those loads as well.
constexpr int kDeepComputeWaves = 8;
constexpr int kDeepLoaderWaves = 4;
constexpr int kDeepThreads = (kDeepComputeWaves + kDeepLoaderWaves) * 64;
constexpr int kXcds = 8;                        // accelerator dies (each with its own L2)
constexpr int kDeepCols = 32;                   // columns per block
constexpr int kDeepPlane = kDeepCols * 4 * 16;  // one digit plane of a block's K step
constexpr int kDeepMaxKs = 4;
constexpr int kDmaBytes = 64 * 16;    // one 16-byte LDS-DMA instruction: 16 bytes per lane
constexpr int kFragBytes = 768 * 16;  // the fragments of one (K step, row tile) unit
constexpr int kDeepLds = 160 * 1024;  // LDS of one workgroup

// Staging order of a block's words (Cin a multiple of 8): the 64-byte run of
// 8 channels (column col, channel group grp) keeps its place, and its 16-byte
// chunk q sits at chunk q ^ deep_swz(col, grp). The conversion's 16-byte reads
// of 16 consecutive lanes (two columns x eight groups, same q) then fall on
// distinct banks.
__device__ __forceinline__ uint32_t deep_swz(uint32_t col, uint32_t grp) { return ((grp >> 1) & 3) ^ (col & 1); }

// LDS address of a shared-memory pointer, as the LDS-DMA instructions take it.
typedef __attribute__((address_space(3))) void *lds_ptr_t;

// The deep kernel's LDS: digit planes [ks][8 planes]; ring staging buffers
// (a block's words in whole LDS-DMA lines, then, streamed, its masks); then
// either the masks of the block being contracted (streamed) or the
// frequency's fragments [ks][row tile][768 items] (resident, whose masks are
// read from global memory). When Cin is not a multiple of 8, 64 spare bytes at
// the end take the reads of a channel group straddling Cin past the last
// column.
struct DeepLds {
    int n_dma, n_mask;
    size_t planes, words, slot, tail, total;
    __host__ __device__ DeepLds(int Cin, int n_ks, int n_ot, bool seeded, bool resident, int ring) {
        n_dma = seeded ? 0 : (kDeepCols * Cin * 8 + kDmaBytes - 1) / kDmaBytes;
        n_mask = 2 * ((n_ot + 1) / 2) * 64;
        planes = (size_t)n_ks * 8 * kDeepPlane;
        words = (size_t)n_dma * kDmaBytes;
        slot = words + (resident ? 0 : (size_t)n_mask * 4);
        tail = resident ? (size_t)n_ks * n_ot * kFragBytes : (size_t)n_mask * 4;
        total = planes + (size_t)ring * slot + tail + (Cin % 8 ? 64 : 0);
    }
};

// SEEDED: seeded input (ensei_homconv_seeded): words j < n come from the
// public stream at conversion and only the b words (column n) are loaded.
// NKS: the layer's K steps of 64 channels (1 to kDeepMaxKs). AL: resident
// fragments. ring: staging buffers (blocks loaded ahead; 1, 2 or 4).
template <bool WIDE_STORE, bool SEEDED, int NKS, bool AL>
__global__ __launch_bounds__(kDeepThreads) void homconv_deep_kernel(HcLayer P, uint64_t delta, int ring) {
    extern __shared__ __attribute__((aligned(16))) uint8_t dlds[];
    constexpr int n_ks = NKS;
    const int n_ot = P.n_ot, Cin = P.Cin, Cout = P.Cout;
    const int n_otp = (n_ot + 1) / 2;
    const int64_t F = P.F, rowlen = (int64_t)P.n + 1;
    const int n_jt = (int)((rowlen + kDeepCols - 1) / kDeepCols);
    const DeepLds L(Cin, n_ks, n_ot, SEEDED, AL, ring);
    const int n_dma = L.n_dma, n_mask = L.n_mask;
    const bool swz = Cin % 8 == 0;
    auto planes = [&](int ks) { return dlds + ks * 8 * kDeepPlane; };
    auto slot = [&](int64_t x) { return dlds + L.planes + (size_t)(x % ring) * L.slot; };  // x: block - blo
    uint8_t *tail = dlds + L.planes + (size_t)ring * L.slot;  // masks in use (streamed) or fragments (resident)
    uint32_t *lds_r = reinterpret_cast<uint32_t *>(tail);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool loader = wave >= kDeepComputeWaves;
    const int g = lane >> 4, l16 = lane & 15, cg = wave & 1, rg = (wave >> 1) & 3;
    const int b_col = cg * 16 + l16;
    const int b_base = plane_slot(b_col, g) * 16;  // this lane's 16 channels of a plane
    const int half = rg & 1, pair_row = rg >> 1;  // 32-row half of row tile 2 otp + pair_row

    // Blocks in (f, b, column) order, so that a frequency's weight fragments
    // serve B * n_jt consecutive blocks. Workgroups are dealt to the XCDs
    // round-robin; renumbering them so that each XCD's workgroups take one
    // contiguous stretch of blocks keeps the fragments of few frequencies in
    // each XCD's L2.
    const int64_t total = P.B * F * n_jt, G = gridDim.x;
    const int64_t wg = G % kXcds == 0 ? (int64_t)(blockIdx.x % kXcds) * (G / kXcds) + blockIdx.x / kXcds
                                      : (int64_t)blockIdx.x;
    const int64_t per = total / G, extra = total % G;
    const int64_t blo = wg * per + (wg < extra ? wg : extra);
    const int64_t bhi = blo + per + (wg < extra ? 1 : 0);
    if (blo >= bhi) return;
    const int64_t nblk = bhi - blo;

    // a block's column block, image and frequency: found by division once
    // per walk, then stepped (the 64-bit divisions are long scalar sequences)
    struct Pos {
        int jt;
        int64_t b, f;
    };
    auto locate = [&](int64_t blk) {
        Pos q;
        q.jt = (int)(blk % n_jt);
        const int64_t fb = blk / n_jt;
        q.b = fb % P.B;
        q.f = fb / P.B;
        return q;
    };
    auto advance = [&](Pos &q, int by) {
        for (int s = 0; s < by; ++s)
            if (++q.jt == n_jt) {
                q.jt = 0;
                if (++q.b == P.B) {
                    q.b = 0;
                    ++q.f;
                }
            }
    };

    if (loader) {
        // Loader waves only issue LDS-DMA loads and wait for their own; their
        // barriers carry no fence, so no wait is added for loads in flight.
        // Group k (the loader waves lw with lw % ring == k, as many as divide
        // evenly) owns the blocks x = k mod ring: it loads block x into slot
        // x % ring once block x - ring has been converted, and waits for it
        // just before the barrier after which x is converted. A group has one
        // block in flight at a time, so that wait is exact.
        const int lw = wave - kDeepComputeWaves;
        const int per_group = kDeepLoaderWaves / ring;
        const int grp = lw % ring, gw = lw / ring;  // group, wave within the group
        const bool act = gw < per_group;
        // 64-byte runs per column; a power of two for 64, 128 and 256 channels
        const uint32_t gpc = (uint32_t)Cin / 8;
        const int gpc_log2 = (gpc & (gpc - 1)) == 0 ? __builtin_ctz(gpc) : -1;
        auto load_block = [&](int64_t x, const Pos &q) {
            const int64_t b = q.b, f = q.f;
            const int jt = q.jt;
            uint8_t *dst = slot(x);
            if (!SEEDED) {
                const __amdgpu_buffer_rsrc_t rs = make_rsrc(
                    uniform_ptr(reinterpret_cast<const uint8_t *>(P.ct_in + (b * F + f) * rowlen * Cin)),
                    (uint32_t)(rowlen * Cin * 8));
                const uint32_t col_off = (uint32_t)((int64_t)jt * kDeepCols * Cin * 8);
                for (int i = gw; i < n_dma; i += per_group) {
                    const uint32_t c = (uint32_t)i * 64 + lane;  // 16-byte chunk of the slot
                    uint32_t gc = c;
                    if (swz) {
                        // run u: column u / gpc, group u % gpc
                        const uint32_t u = c >> 2, col = gpc_log2 >= 0 ? u >> gpc_log2 : u / gpc;
                        gc = (c & ~3u) | ((c & 3u) ^ deep_swz(col, (u - col * gpc) & 7));
                    }
                    const uint32_t d = __builtin_amdgcn_readfirstlane(
                        (uint32_t)(uintptr_t)(lds_ptr_t)(dst + (size_t)i * kDmaBytes));
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)(uintptr_t)d, 16, col_off + gc * 16, 0,
                                                             0, 0);
                }
            }
            if (!AL && jt == n_jt - 1) {
                // masks r[b][o][f], o < Cout (zero past it), 4 bytes per lane
                const __amdgpu_buffer_rsrc_t rr =
                    make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(P.r + b * Cout * F + f)),
                              (uint32_t)(((int64_t)(Cout - 1) * F + 1) * 4));
                for (int i = gw; i * 64 < n_mask; i += per_group) {
                    const int o = i * 64 + lane;
                    const uint32_t d = __builtin_amdgcn_readfirstlane(
                        (uint32_t)(uintptr_t)(lds_ptr_t)(dst + L.words + (size_t)i * 256));
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rr, (lds_ptr_t)(uintptr_t)d, 4,
                                                             o < Cout ? (uint32_t)((int64_t)o * F * 4) : 0x80000000u,
                                                             0, 0, 0);
                }
            }
        };
        // resident: frequency f's fragments, one contiguous run of w_pack
        // (every loader wave takes a share)
        auto load_frags_lds = [&](int64_t f) {
            const uint32_t bytes = (uint32_t)L.tail;
            const __amdgpu_buffer_rsrc_t ra = make_rsrc(
                uniform_ptr(reinterpret_cast<const uint8_t *>(P.w_pack) + f * (int64_t)L.tail), bytes);
            for (int i = lw; i * kDmaBytes < (int)bytes; i += kDeepLoaderWaves) {
                const uint32_t d =
                    __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_ptr_t)(tail + (size_t)i * kDmaBytes));
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_t)(uintptr_t)d, 16,
                                                         (uint32_t)i * kDmaBytes + lane * 16, 0, 0, 0);
            }
        };
        // prologue: the fragments and block 0 landed before the first
        // barrier; blocks 1 .. ring - 1 on their way
        Pos cur = locate(blo);     // block x
        Pos mine = cur;            // the next block this group loads
        advance(mine, grp);
        if (AL) load_frags_lds(cur.f);
        if (act && grp == 0) load_block(0, mine);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        if (act && grp > 0 && grp < nblk) load_block(grp, mine);
        advance(mine, ring);
        __builtin_amdgcn_s_barrier();
        int64_t fprev = cur.f;
        for (int64_t x = 0; x < nblk; ++x) {
            if (AL && cur.f != fprev) {
                // the previous block's phases are done: its frequency's
                // fragments can be replaced while the block is converted
                // (this also waits for the blocks in flight)
                load_frags_lds(cur.f);
                __builtin_amdgcn_s_waitcnt(0x0F70);
            }
            fprev = cur.f;
            __builtin_amdgcn_s_barrier();  // block x converted: its slot is free
            if (x % ring == grp && x + ring < nblk) {
                if (act) load_block(x + ring, mine);
                advance(mine, ring);
            }
            if (act && (x + 1) % ring == grp) __builtin_amdgcn_s_waitcnt(0x0F70);  // block x + 1 landed
            __builtin_amdgcn_s_barrier();  // block x contracted
            advance(cur, 1);
        }
        return;
    }

    // compute waves: block x's words (its ring slot, or the public stream
    // when seeded) -> digit planes, and (streamed) its masks to the masks in
    // use; unit u = (K step, column, 8-channel group)
    auto convert = [&](int64_t x, const Pos &q) {
        const int64_t b = q.b, f = q.f;
        const int jt = q.jt;
        const int col0 = jt * kDeepCols;
        const uint8_t *staging = slot(x);
        if (!AL && jt == n_jt - 1)
            for (int o = tid; o < n_mask; o += kDeepComputeWaves * 64)
                lds_r[o] = reinterpret_cast<const uint32_t *>(staging + L.words)[o];
        for (int u = tid; u < n_ks * 256; u += kDeepComputeWaves * 64) {
            const int uks = u >> 8, col = (u >> 3) & 31, sc = (u >> 1) & 3, h = u & 1;
            const int c0 = uks * 64 + sc * 16 + h * 8;
            uint64_t wd[8];
            if (SEEDED) {
                // words j < n from the public stream, the b word loaded
                const bool on = c0 < Cin && col0 + col < P.n;
                const uint64_t q0 = P.idx0 + (uint64_t)((b * F + f) * Cin + c0);
                uint64_t z = P.seed_a + (q0 * (uint64_t)P.n + (uint64_t)(col0 + col) + 1) * kGamma;
                const uint64_t zstep = (uint64_t)P.n * kGamma;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    wd[i] = on ? splitmix_mix(z) : 0ull;
                    z += zstep;
                }
                if (col0 + col == P.n) {
                    const uint64_t *bw = P.b_in + (b * F + f) * Cin;
#pragma unroll
                    for (int i = 0; i < 8; ++i) wd[i] = c0 + i < Cin ? bw[c0 + i] : 0ull;
                }
            } else if (c0 >= Cin) {
#pragma unroll
                for (int i = 0; i < 8; ++i) wd[i] = 0;
            } else if (swz) {
                const uint32_t run = (uint32_t)(col * (Cin / 8) + c0 / 8), x = deep_swz(col, (c0 / 8) & 7);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const u32x4 t = *reinterpret_cast<const u32x4 *>(staging + (run * 4 + (q ^ x)) * 16);
                    wd[2 * q] = (uint64_t)t.y << 32 | t.x;
                    wd[2 * q + 1] = (uint64_t)t.w << 32 | t.z;
                }
            } else {
                // 8-byte aligned words; a group straddling Cin reads the next
                // column's words (or, past the last column, what follows the
                // words in LDS), which meet zero weights
                const uint64_t *sw = reinterpret_cast<const uint64_t *>(staging) + (col * Cin + c0);
#pragma unroll
                for (int i = 0; i < 8; ++i) wd[i] = sw[i];
            }
            uint32_t lo[8], hi[8], pl[8][2];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint64_t v = wd[i] + 0x8080808080808080ull;
                lo[i] = (uint32_t)v;
                hi[i] = (uint32_t)(v >> 32);
            }
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                transpose4(lo[4 * d], lo[4 * d + 1], lo[4 * d + 2], lo[4 * d + 3], pl[0][d], pl[1][d], pl[2][d],
                           pl[3][d]);
                transpose4(hi[4 * d], hi[4 * d + 1], hi[4 * d + 2], hi[4 * d + 3], pl[4][d], pl[5][d], pl[6][d],
                           pl[7][d]);
            }
            const int pslot = plane_slot(col, sc) * 16 + h * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                *reinterpret_cast<u32x2 *>(planes(uks) + k * kDeepPlane + pslot) =
                    u32x2{pl[k][0] ^ 0x80808080u, pl[k][1] ^ 0x80808080u};
        }
    };

    // streamed: this wave's fragments of unit (f, ks, ot) from the L2, items
    // [limb][row block][lane] (none past the last row tile: the loads return
    // zero); resident: the same items from LDS
    auto load_frags = [&](int64_t f, int ks, int ot, v4i (&A)[3][2]) {
        if (AL) {
            const uint8_t *u = tail + (size_t)(ks * n_ot + (ot < n_ot ? ot : 0)) * kFragBytes;
#pragma unroll
            for (int l = 0; l < 3; ++l)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
                    A[l][rb] = *reinterpret_cast<const v4i *>(u + ((l * 4 + half * 2 + rb) * 64 + lane) * 16);
            return;
        }
        const int64_t unit = (f * n_ks + ks) * n_ot + (ot < n_ot ? ot : 0);
        const __amdgpu_buffer_rsrc_t ra =
            make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(P.w_pack) + unit * kFragBytes),
                      __builtin_amdgcn_readfirstlane(ot < n_ot ? (uint32_t)kFragBytes : 0u));
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const u32x4 t =
                    __builtin_amdgcn_raw_buffer_load_b128(ra, ((l * 4 + half * 2 + rb) * 64 + lane) * 16, 0, 0);
                A[l][rb] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
            }
    };

    Pos cur = locate(blo), nxt = cur;  // block x and block x + 1
    advance(nxt, 1);
    v4i A0[3][2], A1[3][2];
    if (!AL) load_frags(cur.f, 0, pair_row, A0);
    __syncthreads();

    v4i acc[8][2];
    uint64_t res[2][4];
    int64_t f = 0, f_next = 0, b = 0;
    int col0 = 0;
    const uint64_t *oblk = nullptr;
    uint32_t obytes = 0;

    // one phase (row-tile pair otp, K step KS) of the current block. Streamed,
    // it contracts with the fragments in A while those of the next phase load
    // into An; the K step is a compile-time index, so the phases that store
    // are known statically and every wait counts exactly the operations
    // issued after the awaited loads. Resident, A is read from LDS here.
    auto step = [&](auto ks_tag, v4i (&A)[3][2], v4i (&An)[3][2], int otp) {
        constexpr int KS = decltype(ks_tag)::value;
        const int ot = 2 * otp + pair_row;
        if (AL) {
            load_frags(f, KS, ot, A);
        } else {
            // the next phase's fragments (past the block's end: the next block's first)
            if (KS + 1 < NKS)
                load_frags(f, KS + 1, ot, An);
            else if (otp + 1 < n_otp)
                load_frags(f, 0, ot + 2, An);
            else
                load_frags(f_next, 0, pair_row, An);
        }

        const v4i zero = {0, 0, 0, 0};
        if (ot < n_ot) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const v4i Bk = *reinterpret_cast<const v4i *>(planes(KS) + b_base + k * kDeepPlane);
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    if (k + l >= 8) break;
                    const bool first = KS == 0 && (k == 0 || l == 2);
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
                        acc[k + l][rb] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(A[l][rb], Bk, first ? zero : acc[k + l][rb], 0, 0, 0);
                }
            }
        }
        if constexpr (KS == NKS - 1) {
            // the tile's last K step: recombine, HomShare on the b word,
            // store (dropped past the last row tile, so that every such
            // phase issues the same stores)
            if (Cin <= kSmallCin) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        res[rb][i] = recombine<true>(acc[0][rb][i], acc[1][rb][i], acc[2][rb][i], acc[3][rb][i],
                                                     acc[4][rb][i], acc[5][rb][i], acc[6][rb][i], acc[7][rb][i]);
            } else {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        res[rb][i] = recombine<false>(acc[0][rb][i], acc[1][rb][i], acc[2][rb][i], acc[3][rb][i],
                                                      acc[4][rb][i], acc[5][rb][i], acc[6][rb][i], acc[7][rb][i]);
            }
            if (col0 + b_col == P.n && ot < n_ot) {
                const int o0 = ot * 64 + 32 * half + 8 * g;
                const uint32_t *rsrc = P.r + b * Cout * F + f;
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int o = o0 + 4 * rb + i;
                        const uint32_t r = AL ? (o < Cout ? rsrc[(int64_t)o * F] : 0u) : lds_r[o];
                        res[rb][i] += delta * (uint64_t)r;
                    }
            }
            const __amdgpu_buffer_rsrc_t rso = make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(oblk)),
                                                         __builtin_amdgcn_readfirstlane(ot < n_ot ? obytes : 0u));
            store_lane_words<WIDE_STORE, false, 0>(res, rso, b_col, ot * 64 + 32 * half, g, Cout, ot < n_ot);
        }
    };
    // the K steps of one row-tile pair; PAR: which register set holds the
    // first step's fragments
    auto pair = [&](auto par_tag, int otp) {
        constexpr int PAR = decltype(par_tag)::value;
        auto S = [&](auto ks_tag) {
            constexpr int KS = decltype(ks_tag)::value;
            if constexpr (((KS + PAR) & 1) == 0)
                step(ks_tag, A0, A1, otp);
            else
                step(ks_tag, A1, A0, otp);
        };
        S(std::integral_constant<int, 0>{});
        if constexpr (NKS > 1) S(std::integral_constant<int, 1>{});
        if constexpr (NKS > 2) S(std::integral_constant<int, 2>{});
        if constexpr (NKS > 3) S(std::integral_constant<int, 3>{});
    };

    for (int64_t x = 0; x < nblk; ++x) {
        convert(x, cur);
        __syncthreads();  // planes and masks written, the slot free
        b = cur.b;
        f = cur.f;
        f_next = x + 1 < nblk ? nxt.f : cur.f;
        col0 = cur.jt * kDeepCols;
        oblk = P.ct_out + ((b * F + f) * rowlen + col0) * Cout;
        obytes = (uint32_t)((rowlen - col0) * Cout * 8);
        if constexpr (AL || NKS % 2 == 0) {
            for (int otp = 0; otp < n_otp; ++otp) pair(std::integral_constant<int, 0>{}, otp);
        } else {
            int otp = 0;
            for (; otp + 1 < n_otp; otp += 2) {
                pair(std::integral_constant<int, 0>{}, otp);
                pair(std::integral_constant<int, 1>{}, otp + 1);
            }
            if (otp < n_otp) {
                // an odd number of phases: the next block's fragments are in
                // A1; move them to A0 (this waits for them)
                pair(std::integral_constant<int, 0>{}, otp);
#pragma unroll
                for (int l = 0; l < 3; ++l)
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb) A0[l][rb] = A1[l][rb];
            }
        }
        __syncthreads();  // planes read by every compute wave; the next block's words landed
        cur = nxt;
        advance(nxt, 1);
    }
}

// Narrow-input HomConv (Cin <= kNarrowCin, folded weight fragments): with so
// few input channels the launch is a write stream (8 (n+1) Cout bytes out per
// 8 (n+1) Cin in), so nothing here waits on other waves. Each wave walks its
// own units (b, f, row tile ot, 16 columns j): it loads the Cin words of its
// lane's column itself, forms the MFMA's digit operand in registers (lane
// group g needs digit plane s - g of each channel for shift s, which is byte s
// of the balanced digits shifted up by g bytes), and contracts all 64 rows of
// the tile, 32 at a time. The words and mask of the next DEPTH - 1 units are
// in flight meanwhile: a wave's memory counter retires in issue order, so
// waiting for a unit's words also waits for every store issued before them,
// and the depth sets how many units of stores stay in flight. Weight
// fragments stay in registers while the unit's (f, ot) does not change;
// masks are fetched one per lane and handed to the lanes holding the b word
// by a cross-lane read. No LDS, no barrier. SEEDED: seeded input
// (ensei_homconv_seeded): only the b words are loaded, from b_in; the other
// words are generated from the public stream when the unit is converted.
constexpr int kNarrowThreads = 256;
constexpr int kNarrowDepth = 4;  // units in flight per wave

template <int NCH, int DEPTH, bool WIDE_STORE, bool SEEDED>
__global__ __launch_bounds__(kNarrowThreads) void homconv_narrow_kernel(HcLayer P, uint64_t delta) {
    static_assert(NCH % 4 == 0 && NCH <= 16 && DEPTH >= 2, "one 16-channel group");
    constexpr int kWaves = kNarrowThreads / 64;
    constexpr uint64_t kBias = 0x8080808080808080ull;
    const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
    const int64_t W = (int64_t)gridDim.x * kWaves;
    const int64_t gw = (int64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int Cin = P.Cin, Cout = P.Cout, n_ot = P.n_ot;
    const int64_t F = P.F, rowlen = (int64_t)P.n + 1;
    const int n_jb = (int)((rowlen + 15) / 16);
    const int64_t total = P.B * F * n_ot * n_jb;

    // this wave's units: one contiguous range (its output is one contiguous
    // stretch of ct_out when Cout <= 64)
    const int64_t per = total / W, extra = total % W;
    const int64_t u_lo = gw * per + (gw < extra ? gw : extra);
    const int64_t n_units = per + (gw < extra ? 1 : 0);
    if (n_units <= 0) return;

    struct Coord {
        int jb, ot;
        int64_t f, b;
    };
    // units in order: columns fastest, then row tiles, frequencies, images
    auto seek = [&](Coord &c, int64_t u) {
        c.jb = (int)(u % n_jb);
        int64_t x = u / n_jb;
        c.ot = (int)(x % n_ot);
        x /= n_ot;
        c.f = x % F;
        c.b = x / F;
    };
    auto advance = [&](Coord &c) {
        if (++c.jb < n_jb) return;
        c.jb = 0;
        if (++c.ot < n_ot) return;
        c.ot = 0;
        if (++c.f < F) return;
        c.f = 0;
        ++c.b;
    };

    // a unit in flight: the lane's input words and one mask word
    struct Buf {
        uint64_t v[NCH];
        uint32_t r;
    };
    auto issue = [&](const Coord &c, Buf &buf) {
        const uint32_t col = (uint32_t)(c.jb * 16 + l16);
        // seeded: the block of b words, read only by the column block holding column n
        const uint8_t *blk = uniform_ptr(
            SEEDED ? reinterpret_cast<const uint8_t *>(P.b_in + (c.b * F + c.f) * Cin)
                   : reinterpret_cast<const uint8_t *>(P.ct_in + (c.b * F + c.f) * rowlen * Cin));
        const __amdgpu_buffer_rsrc_t rs =
            make_rsrc(blk, SEEDED ? (c.jb == n_jb - 1 ? (uint32_t)(Cin * 8) : 0u) : (uint32_t)(rowlen * Cin * 8));
        // lane group 3 pairs the zero weight limb: it needs no words; columns
        // past n read zero
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const bool want = ch < Cin && g < 3 && (!SEEDED || col == (uint32_t)P.n);
            const uint32_t off = want ? (SEEDED ? (uint32_t)ch * 8 : (col * (uint32_t)Cin + ch) * 8) : 0x80000000u;
            const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
            buf.v[ch] = (uint64_t)t.y << 32 | t.x;
        }
        // masks: only the column block holding the b word (j = n) reads them
        const int o = c.ot * 64 + lane;
        const __amdgpu_buffer_rsrc_t rr =
            make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(P.r + c.b * Cout * F + c.f)),
                      c.jb == n_jb - 1 ? (uint32_t)(((int64_t)(Cout - 1) * F + 1) * 4) : 0u);
        buf.r = __builtin_amdgcn_raw_buffer_load_b32(rr, (int)(o < Cout ? (uint32_t)(o * F * 4) : 0x80000000u), 0, 0);
    };

    Coord cur, nx;
    seek(cur, u_lo);
    v4i A[4];
    int64_t a_key = -1;  // (f, ot) whose weight fragments A holds

    // DEPTH units in flight from the start; the entry issues the same loads
    // and stores as every unit (stores out of range) so that the waits at the
    // loop head see one static count on both incoming paths
    Buf bufs[DEPTH];
    const uint64_t none[2][4] = {};
    const __amdgpu_buffer_rsrc_t no_store = make_rsrc(P.ct_out, 0u);
    nx = cur;
    int64_t issued = 1;
#pragma unroll
    for (int k = 0; k < DEPTH; ++k) {
        if (k > 0 && issued < n_units) {
            advance(nx);
            ++issued;
        }
        issue(nx, bufs[k]);
        store_lane_words<WIDE_STORE, true, kStoreStream>(none, no_store, 0, 0, g, Cout, false);
        store_lane_words<WIDE_STORE, true, kStoreStream>(none, no_store, 0, 0, g, Cout, false);
    }

    auto body = [&](Buf &buf) {
        // a new (f, ot): its weight fragments [row block 4][lane 64] x 16 B
        const int64_t key = cur.f * n_ot + cur.ot;
        if (key != a_key) {
            const __amdgpu_buffer_rsrc_t ra = make_rsrc(
                uniform_ptr(reinterpret_cast<const uint8_t *>(P.w_pack) + key * (int64_t)P.n_items * 16), 4096u);
#pragma unroll
            for (int rbg = 0; rbg < 4; ++rbg) {
                const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(ra, (rbg * 64 + lane) * 16, 0, 0);
                A[rbg] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
            }
            // wait here, on this rare path: left pending past the branch, the
            // fragments would make every unit wait for them (and for all
            // stores issued before them)
            __builtin_amdgcn_s_waitcnt(0);
            a_key = key;
        }
        const uint32_t rv = buf.r;
        if (SEEDED) {
            // words j = col < n of the lane's channels from the public stream
            // (lane group 3 meets the zero limb and needs none)
            const int col = cur.jb * 16 + l16;
            const uint64_t q0 = P.idx0 + (uint64_t)((cur.b * F + cur.f) * Cin);
            uint64_t z = P.seed_a + (q0 * (uint64_t)P.n + (uint64_t)col + 1) * kGamma;
            const uint64_t step = (uint64_t)P.n * kGamma;  // next channel, same word
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const uint64_t a = splitmix_mix(z);
                if (ch < Cin && g < 3 && col < P.n) buf.v[ch] += a;
                z += step;
            }
        }
        // digit operand of shift s: dword q holds digit s - g of channels 4q..4q+3
        uint32_t pl[NCH / 4][8];
#pragma unroll
        for (int q = 0; q < NCH / 4; ++q) {
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t d = ((buf.v[4 * q + i] + kBias) ^ kBias) << (8 * g);
                lo[i] = (uint32_t)d;
                hi[i] = (uint32_t)(d >> 32);
            }
            transpose4(lo[0], lo[1], lo[2], lo[3], pl[q][0], pl[q][1], pl[q][2], pl[q][3]);
            transpose4(hi[0], hi[1], hi[2], hi[3], pl[q][4], pl[q][5], pl[q][6], pl[q][7]);
        }

        // the unit DEPTH ahead reuses this buffer (past the end: reissue the
        // last one, keeping the load count static)
        if (issued < n_units) {
            advance(nx);
            ++issued;
        }
        issue(nx, buf);

        const uint64_t *blk = P.ct_out + ((cur.b * F + cur.f) * rowlen + cur.jb * 16) * Cout;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(uniform_ptr(reinterpret_cast<const uint8_t *>(blk)),
                                                    (uint32_t)((rowlen - cur.jb * 16) * Cout * 8));
        const bool has_b = cur.jb == n_jb - 1;
        const bool b_lane = cur.jb * 16 + l16 == P.n;
        const v4i zero = {0, 0, 0, 0};
#pragma unroll
        for (int rg = 0; rg < 2; ++rg) {
            v4i acc[8][2];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const v4i B = {(int)pl[0][s], NCH > 4 ? (int)pl[NCH > 4 ? 1 : 0][s] : 0,
                               NCH > 8 ? (int)pl[NCH > 8 ? 2 : 0][s] : 0, NCH > 12 ? (int)pl[NCH > 12 ? 3 : 0][s] : 0};
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
                    acc[s][rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[2 * rg + rb], B, zero, 0, 0, 0);
            }
            uint64_t res[2][4];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    res[rb][i] = recombine<true>(acc[0][rb][i], acc[1][rb][i], acc[2][rb][i], acc[3][rb][i],
                                                 acc[4][rb][i], acc[5][rb][i], acc[6][rb][i], acc[7][rb][i]);
            // HomShare: Delta * r on the b word; the mask of tile row x is in lane x
            if (has_b) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t m =
                            (uint32_t)__builtin_amdgcn_ds_bpermute((32 * rg + 8 * g + 4 * rb + i) * 4, (int)rv);
                        if (b_lane) res[rb][i] += delta * (uint64_t)m;
                    }
            }
            store_lane_words<WIDE_STORE, true, kStoreStream>(res, rs, l16, cur.ot * 64 + 32 * rg, g, Cout, true);
        }
        advance(cur);
    };

    for (int64_t it = 0; it < n_units / DEPTH; ++it) {
#pragma unroll
        for (int k = 0; k < DEPTH; ++k) body(bufs[k]);
    }
    const int rem = (int)(n_units % DEPTH);
#pragma unroll
    for (int k = 0; k < DEPTH - 1; ++k)
        if (k < rem) body(bufs[k]);
}

// Weight-fragment item k (16 bytes) of the unit (f, ks, ot): the operand one
// lane of the matrix-core kernel hands the MFMA, in the order its threads load
// and its waves read them.
//   paired (Cin >= 48): 768 items [limb 3][row block 4][lane 64];
//   folded (Cin < 48):  256 * ceil(Cin/16) items [channel group][row block 4][lane 64].
// Lane ln of row block rbg covers tile row 32 (rbg / 2) + 8 (m / 4) + 4 (rbg % 2) + m % 4
// (m = ln % 16), so that after the contraction each output lane holds 8
// consecutive rows; its 16 bytes are one limb of 16 channels: channel group
// 4 ks + ln / 16 and limb `limb` (paired), or channel group sc and limb
// ln / 16 (folded; limb 3 is zero). Digits are the balanced base-256 digits
// of W^ (bytes of W^ + 0x808080, each xor 0x80).
__device__ __forceinline__ int frag_row(int rbg, int m) { return 32 * (rbg >> 1) + 8 * (m >> 2) + 4 * (rbg & 1) + (m & 3); }

// One block per (K step ks, row tile ot) and kPackF consecutive frequencies
// (a "tile" here). The block first reads the tile's 64 x 64 slice of W^ into
// LDS, 16 contiguous bytes (kPackF frequencies) per (row, channel) where W^
// allows it. Then each thread builds the items of one (frequency, 16 channels
// of one row) from LDS: consecutive lanes write consecutive 16-byte items,
// 1 KB per wave store. Reading W^ straight by frequency instead scatters the
// stores (the units of neighbouring frequencies are n_items * 16 bytes apart),
// and every store then writes a piece of a different line. Workgroups are
// renumbered so that each XCD takes a contiguous range of tiles: the tiles
// that share a 128-byte line of W^ read it through one L2.
constexpr int kPackF = 4, kPackThreads = 256;

__global__ __launch_bounds__(kPackThreads) void pack_weights_kernel(const uint32_t *__restrict__ w_hat, int Cout,
                                                                    int Cin, int64_t F, int n_ks, int n_ot,
                                                                    int n_items, int paired, int vec,
                                                                    int8_t *__restrict__ w_pack) {
    __shared__ uint32_t tile[kPackF][64][65];  // [frequency][row][channel], rows padded against bank conflicts
    const int t = threadIdx.x;
    const int per_unit = paired ? 256 : n_items / 4;  // items' producers per unit
    const int64_t f_tiles = (F + kPackF - 1) / kPackF, total = f_tiles * n_ks * n_ot, G = gridDim.x;
    const int64_t wg = G % kXcds == 0 ? (int64_t)(blockIdx.x % kXcds) * (G / kXcds) + blockIdx.x / kXcds
                                      : (int64_t)blockIdx.x;
    const int64_t per = total / G, extra = total % G;
    const int64_t lo = wg * per + (wg < extra ? wg : extra), hi = lo + per + (wg < extra ? 1 : 0);
    for (int64_t T = lo; T < hi; ++T) {
        const int64_t ft = T % f_tiles, u = T / f_tiles;
        const int ot = (int)(u % n_ot), ks = (int)(u / n_ot);
        const int64_t f0 = ft * kPackF;
        const int nf = F - f0 < kPackF ? (int)(F - f0) : kPackF;
        // the slice (rows past Cout and channels past Cin are zero): every
        // thread's loads are issued before any of them is written to LDS
        constexpr int kLoads = 64 * 64 / kPackThreads;
        uint32_t v[kLoads][kPackF];
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int q = t + i * kPackThreads, r = q >> 6, c = q & 63, row = ot * 64 + r, ch = ks * 64 + c;
            const uint32_t *src = w_hat + ((int64_t)row * Cin + ch) * F + f0;
            const bool in = row < Cout && ch < Cin;
            if (vec && nf == kPackF) {
                const uint4 x = in ? *reinterpret_cast<const uint4 *>(src) : make_uint4(0, 0, 0, 0);
                v[i][0] = x.x;
                v[i][1] = x.y;
                v[i][2] = x.z;
                v[i][3] = x.w;
            } else {
#pragma unroll
                for (int k = 0; k < kPackF; ++k) v[i][k] = in && k < nf ? src[k] : 0u;
            }
        }
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int q = t + i * kPackThreads;
#pragma unroll
            for (int k = 0; k < kPackF; ++k) tile[k][q >> 6][q & 63] = v[i][k];
        }
        __syncthreads();
        for (int q = t; q < nf * per_unit; q += kPackThreads) {
            const int fl = q / per_unit, j = q % per_unit;
            // paired: j = (row block, lane), 3 limbs at k = limb * 256 + j;
            // folded: j = (group, row block, m), 4 slots at k = group * 256 + rbg * 64 + slot * 16 + m
            const int rbg = paired ? (j >> 6) : ((j >> 4) & 3);
            const int m = j & 15;
            const int lg = paired ? ((j & 63) >> 4) : (j >> 6);  // 16-channel group within the K step
            const int lr = frag_row(rbg, m);
            uint32_t dig[4][4] = {};
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const uint32_t uu = (tile[fl][lr][lg * 16 + c] + 0x808080u) ^ 0x808080u;  // balanced digits (byte 3 is 0)
#pragma unroll
                for (int l = 0; l < 4; ++l) dig[l][c >> 2] |= ((uu >> (8 * l)) & 0xffu) << (8 * (c & 3));
            }
            const int64_t unit = ((f0 + fl) * n_ks + ks) * n_ot + ot;
            uint4 *dst = reinterpret_cast<uint4 *>(w_pack) + unit * n_items;
            if (paired) {
#pragma unroll
                for (int l = 0; l < 3; ++l) dst[l * 256 + j] = make_uint4(dig[l][0], dig[l][1], dig[l][2], dig[l][3]);
            } else {
                const int k0 = (j >> 6) * 256 + rbg * 64 + m;
#pragma unroll
                for (int l = 0; l < 4; ++l) dst[k0 + l * 16] = make_uint4(dig[l][0], dig[l][1], dig[l][2], dig[l][3]);
            }
        }
        __syncthreads();  // the slice is rewritten for the next tile
    }
}

int homconv_sizes(int64_t batch, int Cin, int Cout, int64_t F, int n) {
    if (batch <= 0 || Cin <= 0 || Cout <= 0 || F <= 0 || n <= 0) return ENSEI_ERR_ARG;
    if (Cin > ENSEI_MAX_CIN || Cout > ENSEI_MAX_COUT || n > ENSEI_MAX_LWE_N || F > (1 << 20)) return ENSEI_ERR_LIMIT;
    // one (b, f) block of either side is addressed with 32-bit byte offsets
    if ((int64_t)(n + 1) * (Cin > Cout ? Cin : Cout) * 8 > 0x7fffffff) return ENSEI_ERR_LIMIT;
    if ((int64_t)Cout * F * 4 > 0x7fffffff) return ENSEI_ERR_LIMIT;  // one image's masks, likewise
    return ENSEI_OK;
}

// seeded: ct_in holds only the b words, [B][F][Cin]
static int check_homconv(const ensei_ctx *ctx, const void *ct_in, const void *w, const void *r, int64_t batch,
                         int Cin, int Cout, int64_t F, int n, const void *ct_out, size_t wbytes, bool seeded = false) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!ct_in || !w || !r || !ct_out) return ENSEI_ERR_ARG;
    st = homconv_sizes(batch, Cin, Cout, F, n);
    if (st) return st;
    if (((uintptr_t)ct_in & 7) || ((uintptr_t)ct_out & 7) || ((uintptr_t)r & 3)) return ENSEI_ERR_ALIGN;
    const size_t inb = (size_t)batch * Cin * F * (seeded ? 1 : n + 1) * 8, outb = (size_t)batch * Cout * F * (n + 1) * 8;
    if (overlaps(ct_out, outb, ct_in, inb) || overlaps(ct_out, outb, w, wbytes) ||
        overlaps(ct_out, outb, r, (size_t)batch * Cout * F * 4))
        return ENSEI_ERR_OVERLAP;
    return ENSEI_OK;
}

size_t wpack_bytes_as(int Cout, int Cin, int64_t F, bool paired) {
    if (Cout <= 0 || Cin <= 0 || F <= 0) return 0;
    return (size_t)F * ((Cin + 63) / 64) * ((Cout + 63) / 64) * frag_items(Cin, paired) * 16;
}

int pack_weights_as(const ensei_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F, bool paired,
                    int8_t *w_pack, hipStream_t stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!w_hat || !w_pack || Cout <= 0 || Cin <= 0 || F <= 0) return ENSEI_ERR_ARG;
    if (Cin > ENSEI_MAX_CIN || Cout > ENSEI_MAX_COUT || F > (1 << 20)) return ENSEI_ERR_LIMIT;
    if (!paired && Cin >= 64) return ENSEI_ERR_ARG;  // the folded layout holds one 64-channel step
    if (((uintptr_t)w_hat & 3) || ((uintptr_t)w_pack & 15)) return ENSEI_ERR_ALIGN;
    if (overlaps(w_pack, wpack_bytes_as(Cout, Cin, F, paired), w_hat, (size_t)Cout * Cin * F * 4))
        return ENSEI_ERR_OVERLAP;
    const int n_ks = (Cin + 63) / 64, n_ot = (Cout + 63) / 64, n_items = frag_items(Cin, paired);
    const int64_t tiles = (F + kPackF - 1) / kPackF * n_ks * n_ot;
    // two resident workgroups per CU; a multiple of the XCD count when there are enough tiles
    int64_t blocks = 2 * (int64_t)ctx->num_cus;
    if (tiles < blocks) blocks = tiles >= kXcds ? tiles / kXcds * kXcds : tiles;
    const int vec = ((uintptr_t)w_hat & 15) == 0 && F % kPackF == 0;
    hipLaunchKernelGGL(pack_weights_kernel, dim3((unsigned)blocks), dim3(kPackThreads), 0, stream, w_hat, Cout, Cin, F,
                       n_ks, n_ot, n_items, (int)paired, vec, w_pack);
    return launch_status();
}

int homconv_problem(const ensei_ctx *ctx, HcLayer *P, const uint64_t *ct_in, const int8_t *w_pack, const uint32_t *r,
                    int64_t B, int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, size_t wbytes, bool seeded) {
    int st = check_homconv(ctx, ct_in, w_pack, r, B, Cin, Cout, F, n, ct_out, wbytes, seeded);
    if (st) return st;
    if ((uintptr_t)w_pack & 15) return ENSEI_ERR_ALIGN;
    P->ct_in = seeded ? nullptr : ct_in;
    P->b_in = seeded ? ct_in : nullptr;
    P->seed_a = P->idx0 = 0;
    P->w_pack = w_pack;
    P->r = r;
    P->ct_out = ct_out;
    P->F = F;
    P->B = B;
    P->Cin = Cin;
    P->Cout = Cout;
    P->n = n;
    P->n_ot = (Cout + 63) / 64;
    P->n_jt = (n + 1 + 63) / 64;
    P->n_ks = (Cin + 63) / 64;
    P->n_items = frag_items(Cin, Cin >= kPairedCin);
    P->tile0 = 0;
    P->n_tiles = B * F * P->n_jt * P->n_ot;
    P->pad = 0;
    return ENSEI_OK;
}

// Narrow kernel launch: enough 4-wave workgroups to fill every CU at the
// kernel's occupancy (each wave walks its own contiguous range of units).
template <int NCH, bool SEEDED>
static int launch_narrow(const ensei_ctx *ctx, const HcLayer &P, HcSchedule sched, hipStream_t stream) {
    const bool wide = P.Cout % 2 == 0;
    auto kernel = wide ? homconv_narrow_kernel<NCH, kNarrowDepth, true, SEEDED>
                       : homconv_narrow_kernel<NCH, kNarrowDepth, false, SEEDED>;
    static std::atomic<int> resident[kMaxDevices][2];  // workgroups per CU, by device and store width
    const bool cached = ctx->device < kMaxDevices;
    int per_cu = cached ? resident[ctx->device][wide].load(std::memory_order_relaxed) : 0;
    if (per_cu == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kNarrowThreads, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (cached) resident[ctx->device][wide].store(per_cu, std::memory_order_relaxed);
    }
    const int64_t units = P.B * P.F * P.n_ot * ((P.n + 1 + 15) / 16);
    int64_t blocks = sched.blocks > 0 ? sched.blocks : (int64_t)ctx->num_cus * per_cu;
    const int64_t needed = (units + kNarrowThreads / 64 - 1) / (kNarrowThreads / 64);
    if (blocks > needed) blocks = needed;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kNarrowThreads), 0, stream, P, ctx->delta);
    return launch_status();
}

// Deep kernel launch, if the layer suits it (homconv_deep_fits). Returns
// ENSEI_ERR_LIMIT (nothing launched) otherwise.
bool homconv_deep_fits(const HcLayer &P, bool seeded) {
    // all K steps of a block in LDS beside a staging buffer, several row
    // tiles and (plain input) at least four (row tile, K step) pairs per block
    // to share the conversion (the 64 -> 128 layer, two pairs, is faster on
    // the streaming kernel: 700-750 against 930 us); seeded input takes every
    // layer with two or more row tiles (the stream is generated once per
    // block, not per row tile)
    return P.Cin >= kPairedCin && P.n_ks <= kDeepMaxKs && P.n_ot >= 2 && (seeded || P.n_ot * P.n_ks >= 4) &&
           DeepLds(P.Cin, P.n_ks, P.n_ot, seeded, false, 1).total <= (size_t)kDeepLds;
}

template <bool SEEDED>
static int launch_deep(const ensei_ctx *ctx, const HcLayer &P, hipStream_t stream) {
    if (!homconv_deep_fits(P, SEEDED)) return ENSEI_ERR_LIMIT;
    // resident fragments when the frequency's set fits beside the rest; then
    // as many staging buffers as fit (1, 2 or 4). With streamed fragments
    // one: more blocks in flight lengthen the fragment loads' round trips
    // more than they gain.
    const bool al = DeepLds(P.Cin, P.n_ks, P.n_ot, SEEDED, true, 1).total <= (size_t)kDeepLds;
    int ring = 1;
    if (al)
        for (int r : {4, 2})
            if (DeepLds(P.Cin, P.n_ks, P.n_ot, SEEDED, true, r).total <= (size_t)kDeepLds) {
                ring = r;
                break;
            }
    const size_t lds = DeepLds(P.Cin, P.n_ks, P.n_ot, SEEDED, al, ring).total;
    const bool wide = P.Cout % 2 == 0;
    using Kern = void (*)(HcLayer, uint64_t, int);
    static const Kern kernels[2][2][kDeepMaxKs] = {
        {{homconv_deep_kernel<false, SEEDED, 1, false>, homconv_deep_kernel<false, SEEDED, 2, false>,
          homconv_deep_kernel<false, SEEDED, 3, false>, homconv_deep_kernel<false, SEEDED, 4, false>},
         {homconv_deep_kernel<false, SEEDED, 1, true>, homconv_deep_kernel<false, SEEDED, 2, true>,
          homconv_deep_kernel<false, SEEDED, 3, true>, homconv_deep_kernel<false, SEEDED, 4, true>}},
        {{homconv_deep_kernel<true, SEEDED, 1, false>, homconv_deep_kernel<true, SEEDED, 2, false>,
          homconv_deep_kernel<true, SEEDED, 3, false>, homconv_deep_kernel<true, SEEDED, 4, false>},
         {homconv_deep_kernel<true, SEEDED, 1, true>, homconv_deep_kernel<true, SEEDED, 2, true>,
          homconv_deep_kernel<true, SEEDED, 3, true>, homconv_deep_kernel<true, SEEDED, 4, true>}}};
    const Kern kernel = kernels[wide][al][P.n_ks - 1];
    // dynamic-LDS limit raised, by device, store width, fragments and K steps
    static std::atomic<bool> attr[kMaxDevices][2][2][kDeepMaxKs];
    const bool cached = ctx->device < kMaxDevices;
    if (!cached || !attr[ctx->device][wide][al][P.n_ks - 1].load(std::memory_order_acquire)) {
        if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kDeepLds) !=
            hipSuccess)
            return ENSEI_ERR_HIP;
        if (cached) attr[ctx->device][wide][al][P.n_ks - 1].store(true, std::memory_order_release);
    }
    // one resident workgroup per CU
    const int64_t blocks_total = P.B * P.F * ((P.n + 1 + kDeepCols - 1) / kDeepCols);
    const int64_t grid = blocks_total < (int64_t)ctx->num_cus ? blocks_total : (int64_t)ctx->num_cus;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(kDeepThreads), lds, stream, P, ctx->delta, ring);
    return launch_status();
}

// The streaming kernel for a launch's layout: paired or folded limbs, even or
// odd Cout, one problem or a table of them, plain or seeded input.
template <bool MULTI, bool SEEDED>
static void launch_streaming(const ensei_ctx *ctx, const HcLayer *problems, const HcLayer *dev_table, int nlayers,
                             bool paired, bool wide, int64_t blocks, int64_t total, int64_t chunk, hipStream_t stream) {
    if (MULTI) {  // multi-problem launches use paired fragments
        auto kernel = wide ? homconv_mfma_kernel<true, true, true, SEEDED> : homconv_mfma_kernel<true, false, true, SEEDED>;
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kHcThreads), 0, stream, problems[0], dev_table, nlayers,
                           total, chunk, ctx->delta);
        return;
    }
    // one limb pair per MFMA once the 64-channel K steps are full enough;
    // limbs folded into K for narrow inputs
    auto kernel = paired ? (wide ? homconv_mfma_kernel<true, true, false, SEEDED>
                                 : homconv_mfma_kernel<true, false, false, SEEDED>)
                         : (wide ? homconv_mfma_kernel<false, true, false, SEEDED>
                                 : homconv_mfma_kernel<false, false, false, SEEDED>);
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kHcThreads), 0, stream, problems[0], dev_table, 1, total,
                       chunk, ctx->delta);
}

int homconv_launch(const ensei_ctx *ctx, const HcLayer *problems, const HcLayer *dev_table, int nlayers, bool paired,
                   HcSchedule sched, hipStream_t stream, bool seeded) {
    if (nlayers < 1 || (nlayers > 1 && (!dev_table || !paired))) return ENSEI_ERR_ARG;
    if (sched.chunk < 0) return ENSEI_ERR_ARG;
    if (nlayers == 1 && paired && sched.blocks == 0) {
        const int rc = seeded ? launch_deep<true>(ctx, problems[0], stream) : launch_deep<false>(ctx, problems[0], stream);
        if (rc != ENSEI_ERR_LIMIT) return rc;
    }
    if (nlayers == 1 && !paired && problems[0].Cin <= kNarrowCin) {
        const bool four = problems[0].Cin <= 4;
        if (seeded)
            return four ? launch_narrow<4, true>(ctx, problems[0], sched, stream)
                        : launch_narrow<8, true>(ctx, problems[0], sched, stream);
        return four ? launch_narrow<4, false>(ctx, problems[0], sched, stream)
                    : launch_narrow<8, false>(ctx, problems[0], sched, stream);
    }
    int64_t total = 0;
    bool wide = true;
    for (int L = 0; L < nlayers; ++L) {
        total += problems[L].n_tiles;
        wide = wide && problems[L].Cout % 2 == 0;
    }
    // persistent grid: at most one resident 8-wave workgroup per CU
    int64_t blocks = sched.blocks > 0 ? sched.blocks : ctx->num_cus;
    if (blocks > ctx->num_cus) blocks = ctx->num_cus;
    if (sched.chunk == 0 && total < blocks) blocks = total;
    const bool multi = nlayers > 1;
    if (multi && seeded)
        launch_streaming<true, true>(ctx, problems, dev_table, nlayers, paired, wide, blocks, total, sched.chunk, stream);
    else if (multi)
        launch_streaming<true, false>(ctx, problems, dev_table, nlayers, paired, wide, blocks, total, sched.chunk, stream);
    else if (seeded)
        launch_streaming<false, true>(ctx, problems, dev_table, 1, paired, wide, blocks, total, sched.chunk, stream);
    else
        launch_streaming<false, false>(ctx, problems, dev_table, 1, paired, wide, blocks, total, sched.chunk, stream);
    return launch_status();
}

}  // namespace ensei

using namespace ensei;

extern "C" {

size_t ensei_wpack_bytes(int Cout, int Cin, int64_t F) { return wpack_bytes_as(Cout, Cin, F, Cin >= kPairedCin); }

int ensei_pack_weights(ensei_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F, int8_t *w_pack,
                       void *stream) {
    return pack_weights_as(ctx, w_hat, Cout, Cin, F, Cin >= kPairedCin, w_pack, (hipStream_t)stream);
}

int ensei_homconv(ensei_ctx *ctx, const uint64_t *ct_in, const int8_t *w_pack, const uint32_t *r, int64_t batch,
                  int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, void *stream) {
    HcLayer P;
    int st = homconv_problem(ctx, &P, ct_in, w_pack, r, batch, Cin, Cout, F, n, ct_out,
                             ensei_wpack_bytes(Cout, Cin, F));
    if (st) return st;
    return homconv_launch(ctx, &P, nullptr, 1, Cin >= kPairedCin, HcSchedule{0, 0}, (hipStream_t)stream);
}

int ensei_homconv_seeded(ensei_ctx *ctx, const uint64_t *b_in, uint64_t seed_a, uint64_t ct_index0,
                         const int8_t *w_pack, const uint32_t *r, int64_t batch, int Cin, int Cout, int64_t F, int n,
                         uint64_t *ct_out, void *stream) {
    HcLayer P;
    int st = homconv_problem(ctx, &P, b_in, w_pack, r, batch, Cin, Cout, F, n, ct_out,
                             ensei_wpack_bytes(Cout, Cin, F), true);
    if (st) return st;
    P.seed_a = seed_a;
    P.idx0 = ct_index0;
    return homconv_launch(ctx, &P, nullptr, 1, Cin >= kPairedCin, HcSchedule{0, 0}, (hipStream_t)stream, true);
}

}  // extern "C"
