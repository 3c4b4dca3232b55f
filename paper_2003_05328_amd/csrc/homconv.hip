// HomConv: for every (image b, frequency f) an exact integer contraction
//   ct_out[b][:, f, :] = W^_f (Cout x Cin) . ct_in[b][:, f, :] (Cin x (n+1))  mod 2^64
// plus Delta * r[b][o][f] on the b word (HomShare).
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
//   One MFMA's 64-long K dimension holds 16 channels x 4 limb slots
//   (slot l < 3 pairs limb w_l with ciphertext digit plane s - l; slot 3 is
//   zero), so one instruction per shift s covers all three limbs of 16
//   channels.
//
// Work decomposition: one workgroup (4 waves) per output tile of
// (b, f, 16*RB rows o, 64 columns j); the b column j = n is simply the last
// column and gets Delta*r in the epilogue. Per 64 input channels the waves
// stream the 64 x 64 ciphertext words from HBM (each wave one 16-channel
// group, lanes along j so every load moves 512 contiguous bytes), convert
// them to digit planes with byte permutes, and store the planes in LDS as
// [plane][channel group][column][16 channel bytes], which makes both the
// 16-byte LDS writes and the MFMA B-operand reads conflict free. Each wave
// then owns 16 columns x 16*RB rows and keeps the eight shift accumulators
// in registers; the epilogue recombines them into u64 words and writes
// ct_out with 128-byte row segments. Tiles are assigned XCD by XCD so tiles
// that share (b, f) (hence W^_f and, for several row tiles, ct_in) run on
// the same L2.
#include "ensei_internal.hpp"

namespace ensei {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kPlaneBytes = 4 * 64 * 16;  // 4 channel groups x 64 columns x 16 bytes

// Bijective block -> tile map giving XCD x (= block % 8) a contiguous tile range.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t nblk) {
    const int64_t q = nblk >> 3, rem = nblk & 7, x = bid & 7, k = bid >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

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

// Store of one u64 per lane through a raw buffer descriptor covering
// [base, base + nbytes): writes at or past nbytes are dropped by the hardware
// range check, so a store instruction is issued (and counted) even when none
// of its lanes has anything to write. base and nbytes are wave-uniform.
__device__ __forceinline__ void store_u64_bounded(uint8_t *base, uint32_t nbytes, uint32_t off, uint64_t v) {
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)nbytes, 0x00020000);
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 d = {(unsigned)v, (unsigned)(v >> 32)};
    __builtin_amdgcn_raw_buffer_store_b64(d, rsrc, (int)off, 0, 0);
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

// Persistent, software-pipelined HomConv. Work units are (tile, K step)
// pairs, a K step being 64 input channels, a tile (b, f, 16*RB rows, 64
// columns); each workgroup walks a contiguous range of tiles with row tiles
// fastest, so consecutive units reuse the same ciphertext words and weight
// fragments from L2. Everything a unit needs from HBM - its 64 x 64 words,
// its weight fragments and its masks - is loaded one unit ahead into
// registers: while the MFMAs of the current unit run, the next unit's data is
// in flight. Loads are unconditional: clamped channels meet zero weights
// (the packed weights are zero-padded) and clamped columns are never stored,
// so nothing needs masking. Addresses are a wave-uniform 64-bit base plus a
// 32-bit lane offset, which keeps 64-bit multiplies out of the loop.
// Finished tiles are staged in LDS and written one contiguous row segment per
// store instruction, issued after the next prefetch and in the same number
// every iteration: the vector-memory counter retires in order, so the wait for
// the prefetched words then never waits for these stores.
template <int RB>
__global__ __launch_bounds__(256) void homconv_mfma_kernel(const uint64_t *__restrict__ ct_in,
                                                           const int8_t *__restrict__ w_pack,
                                                           const uint32_t *__restrict__ r, int Cin, int Cout,
                                                           int64_t F, int n, uint64_t delta,
                                                           uint64_t *__restrict__ ct_out, int n_ot, int n_jt, int SC,
                                                           int Cout16, int64_t n_tiles, int n_ks) {
    constexpr int kA = 4 * RB * 64 * 16;  // weight fragments of one unit: [sc][rb][lane][16 B]
    constexpr int kOutStride = 65;        // u64 per staged output row (64 columns + pad)
    constexpr int kOut = 16 * RB * kOutStride * 8;
    // digit planes k = -2..7 at (k + 2) * kPlaneBytes (planes -2, -1 zero), then
    // the unit's weight fragments, its 16*RB masks, and the finished tile
    __shared__ __attribute__((aligned(16))) uint8_t lds[10 * kPlaneBytes + kA + 64 * 4 + kOut];
    uint8_t *lds_a = lds + 10 * kPlaneBytes;
    uint32_t *lds_r = reinterpret_cast<uint32_t *>(lds + 10 * kPlaneBytes + kA);
    uint64_t *lds_out = reinterpret_cast<uint64_t *>(lds + 10 * kPlaneBytes + kA + 64 * 4);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t rowlen = (int64_t)n + 1;
    const int64_t ch_bytes = F * rowlen * 8;    // one input channel
    const int64_t orow_bytes = F * rowlen * 8;  // one output row o

    // this block's contiguous tile range
    const int64_t per = n_tiles / gridDim.x, extra = n_tiles % gridDim.x;
    const int64_t t0 = blockIdx.x * per + (blockIdx.x < extra ? blockIdx.x : extra);
    int64_t todo = per + (blockIdx.x < extra ? 1 : 0);
    if (todo == 0) return;

    for (int i = tid; i < 2 * kPlaneBytes / 16; i += 256) reinterpret_cast<uint4 *>(lds)[i] = make_uint4(0, 0, 0, 0);

    const int b_base = (g == 3 ? 1 : 2 - g) * kPlaneBytes;  // B: plane s - g, zero plane for slot 3
    const int b_step = g == 3 ? 0 : kPlaneBytes;

    // weight-fragment items k = tid + 256 j: sc = k / (64 RB) and rb are
    // wave-uniform, the MFMA lane is k % 64
    uint32_t a_lane_off[RB];
    int a_sc[RB], a_rb[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        const int k = tid + 256 * j;
        const int ln = k % 64;
        const int slot = (ln >> 4) < 3 ? (ln >> 4) : 2;  // slot 3 meets the zero B plane
        a_lane_off[j] = (uint32_t)((ln & 15) * 48 + slot * 16);
        a_sc[j] = __builtin_amdgcn_readfirstlane(k / (64 * RB));
        a_rb[j] = __builtin_amdgcn_readfirstlane((k / 64) % RB);
    }
    const int r_row = tid & (16 * RB - 1);

    // unit coordinates (wave-uniform), advanced incrementally
    int64_t t = t0;
    int ot = (int)(t % n_ot);
    t /= n_ot;
    int jt = (int)(t % n_jt);
    t /= n_jt;
    int64_t f = t % F, b = t / F;
    int ks = 0;

    uint64_t pre[16];
    v4i pre_a[RB];
    uint32_t pre_r;
    auto issue = [&](int u_ot, int u_jt, int64_t u_f, int64_t u_b, int u_ks) {
        const int jl = u_jt * 64 + lane;
        const uint32_t col_off = (uint32_t)((jl <= n ? jl : n) * 8);
        const int ch0 = u_ks * 64 + wave * 16;
        const int lastq = Cin - 1 - ch0;  // channels past Cin re-read channel Cin-1
        const uint8_t *src = uniform_ptr(reinterpret_cast<const uint8_t *>(ct_in) +
                                         ((u_b * Cin) * F + u_f) * rowlen * 8 + (int64_t)ch0 * ch_bytes);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            pre[q] = load_global<uint64_t>(uniform_ptr(src + (int64_t)(q < lastq ? q : lastq) * ch_bytes), col_off);
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            int scg = u_ks * 4 + a_sc[j];
            scg = scg < SC ? scg : SC - 1;
            // a row block past Cout16 (only whole blocks can be) re-reads the last
            // real block: its rows are computed but never stored
            int row = u_ot * 16 * RB + a_rb[j] * 16;
            row = row < Cout16 ? row : Cout16 - 16;
            const uint8_t *wa = uniform_ptr(reinterpret_cast<const uint8_t *>(w_pack) +
                                            (((int64_t)u_f * SC + scg) * Cout16 + row) * 48);
            pre_a[j] = load_global<v4i>(wa, a_lane_off[j]);
        }
        int o = u_ot * 16 * RB + r_row;
        o = o < Cout ? o : Cout - 1;
        pre_r = r[(u_b * Cout + o) * F + u_f];
    };

    issue(ot, jt, f, b, 0);
    v4i acc[8][RB];
    uint64_t res[RB][4] = {};
    bool have_out = false;  // res holds a finished tile not yet stored
    uint8_t *out_base = reinterpret_cast<uint8_t *>(ct_out);
    uint32_t out_nbytes = 0;
    int out_rows = 0;

    // one store per staged row (wave + 4k); rows past out_rows, columns past n
    // and iterations without a finished tile are dropped by the bounds
    auto store_tile = [&](bool valid) {
#pragma unroll
        for (int k = 0; k < 4 * RB; ++k) {
            const int row = wave + 4 * k;
            store_u64_bounded(out_base + row * orow_bytes, valid && row < out_rows ? out_nbytes : 0u,
                              (uint32_t)lane * 8, lds_out[row * kOutStride + lane]);
        }
    };

    // the loop issues prefetch loads followed by tile stores; the entry issues
    // the same sequence (stores fully out of bounds, hence dropped) so that the
    // waits at the loop head see one static count on both incoming paths
    store_tile(false);

    while (true) {
        const int o0 = ot * 16 * RB, j0 = jt * 64;
        const bool last_ks = ks == n_ks - 1;

        // digit planes of this unit's words
        uint32_t pl[8][4];
        {
            uint32_t lo[16], hi[16];
#pragma unroll
            for (int qq = 0; qq < 16; ++qq) {
                const uint64_t v = pre[qq] + 0x8080808080808080ull;
                lo[qq] = (uint32_t)v;
                hi[qq] = (uint32_t)(v >> 32);
            }
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                transpose4(lo[4 * d], lo[4 * d + 1], lo[4 * d + 2], lo[4 * d + 3], pl[0][d], pl[1][d], pl[2][d],
                           pl[3][d]);
                transpose4(hi[4 * d], hi[4 * d + 1], hi[4 * d + 2], hi[4 * d + 3], pl[4][d], pl[5][d], pl[6][d],
                           pl[7][d]);
            }
        }
        __syncthreads();  // the previous unit's MFMA reads and staged-tile reads are done
#pragma unroll
        for (int k = 0; k < 8; ++k)
            *reinterpret_cast<uint4 *>(lds + (k + 2) * kPlaneBytes + (wave * 64 + lane) * 16) =
                make_uint4(pl[k][0] ^ 0x80808080u, pl[k][1] ^ 0x80808080u, pl[k][2] ^ 0x80808080u,
                           pl[k][3] ^ 0x80808080u);
#pragma unroll
        for (int j = 0; j < RB; ++j) reinterpret_cast<v4i *>(lds_a)[tid + 256 * j] = pre_a[j];
        if (tid < 16 * RB) lds_r[tid] = pre_r;
        // the finished tile: lane holds rows rb*16 + 4g + i of column 16*wave + l16
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) lds_out[(rb * 16 + 4 * g + i) * kOutStride + wave * 16 + l16] = res[rb][i];
        __syncthreads();

        // advance to the next unit and put its data in flight (the last unit
        // reloads itself so that the number of loads, and every wait, is static)
        const int c_ks = ks;
        const int64_t c_f = f, c_b = b;
        const bool more = !(last_ks && todo == 1);
        if (more) {
            if (!last_ks) {
                ++ks;
            } else {
                ks = 0;
                --todo;
                if (++ot == n_ot) {
                    ot = 0;
                    if (++jt == n_jt) {
                        jt = 0;
                        if (++f == F) {
                            f = 0;
                            ++b;
                        }
                    }
                }
            }
        }
        issue(ot, jt, f, b, ks);
        store_tile(have_out);
        have_out = false;

        if (c_ks == 0) {
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc[s][rb] = v4i{0, 0, 0, 0};
        }
#pragma unroll
        for (int sc = 0; sc < 4; ++sc) {
            if (c_ks * 4 + sc >= SC) break;
            v4i Ar[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) Ar[rb] = reinterpret_cast<const v4i *>(lds_a)[(sc * RB + rb) * 64 + lane];
            const uint8_t *bp = lds + b_base + (sc * 64 + wave * 16 + l16) * 16;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const v4i B = *reinterpret_cast<const v4i *>(bp + s * b_step);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    acc[s][rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Ar[rb], B, acc[s][rb], 0, 0, 0);
            }
        }

        if (last_ks) {
            // recombine: lane holds rows 4*g + i (i < 4) of column l16 in each row block
            const int jc = j0 + wave * 16 + l16;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t lo64 = (int64_t)acc[0][rb][i] + (int64_t)acc[1][rb][i] * 256 +
                                         (int64_t)acc[2][rb][i] * 65536 + (int64_t)acc[3][rb][i] * 16777216;
                    const uint32_t hi32 = (uint32_t)acc[4][rb][i] + ((uint32_t)acc[5][rb][i] << 8) +
                                          ((uint32_t)acc[6][rb][i] << 16) + ((uint32_t)acc[7][rb][i] << 24);
                    uint64_t v = (uint64_t)lo64 + ((uint64_t)hi32 << 32);
                    if (jc == n) v += delta * (uint64_t)lds_r[rb * 16 + 4 * g + i];
                    res[rb][i] = v;
                }
            have_out = true;
            out_rows = Cout - o0;
            out_nbytes = (uint32_t)((n + 1 - j0) * 8);
            out_base = reinterpret_cast<uint8_t *>(ct_out + ((c_b * Cout + o0) * F + c_f) * rowlen + j0);
        }
        if (!more) break;
    }
    if (have_out) {
        __syncthreads();  // every wave is done reading the previously staged tile
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) lds_out[(rb * 16 + 4 * g + i) * kOutStride + wave * 16 + l16] = res[rb][i];
        __syncthreads();
        store_tile(true);
    }
}

// w_hat [Cout][Cin][F] -> w_pack [F][SC][Cout16][3][16]: balanced base-256 digits.
__global__ void pack_weights_kernel(const uint32_t *__restrict__ w_hat, int Cout, int Cin, int64_t F, int SC,
                                    int Cout16, int8_t *__restrict__ w_pack) {
    const int64_t total = F * SC * Cout16;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = idx % F;
        const int64_t rest = idx / F;
        const int o = (int)(rest % Cout16), sc = (int)(rest / Cout16);
        uint32_t dig[3][4] = {};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int i = sc * 16 + c;
            uint32_t w = 0;
            if (o < Cout && i < Cin) w = w_hat[((int64_t)o * Cin + i) * F + f];
            const uint32_t u = (w + 0x808080u) ^ 0x808080u;  // balanced digits as bytes
#pragma unroll
            for (int l = 0; l < 3; ++l) dig[l][c >> 2] |= ((u >> (8 * l)) & 0xffu) << (8 * (c & 3));
        }
        uint4 *dst = reinterpret_cast<uint4 *>(w_pack + (((f * SC + sc) * Cout16 + o) * 3) * 16);
#pragma unroll
        for (int l = 0; l < 3; ++l) dst[l] = make_uint4(dig[l][0], dig[l][1], dig[l][2], dig[l][3]);
    }
}

// Vector-ALU HomConv: one thread per column j, TO consecutive rows o in
// registers; W^[o][i][f] is uniform across the workgroup (scalar loads).
template <int TO>
__global__ __launch_bounds__(256) void homconv_valu_kernel(const uint64_t *__restrict__ ct_in,
                                                           const uint32_t *__restrict__ w_hat,
                                                           const uint32_t *__restrict__ r, int Cin, int Cout,
                                                           int64_t F, int n, uint64_t delta,
                                                           uint64_t *__restrict__ ct_out, int n_jb, int n_ot) {
    int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int jb = (int)(t % n_jb);
    t /= n_jb;
    const int ot = (int)(t % n_ot);
    t /= n_ot;
    const int64_t f = t % F, b = t / F;
    const int j = jb * 256 + threadIdx.x;
    if (j > n) return;
    const int o0 = ot * TO;
    const int64_t rowlen = (int64_t)n + 1;
    uint64_t acc[TO];
#pragma unroll
    for (int k = 0; k < TO; ++k) acc[k] = 0;
    const uint64_t *src = ct_in + (b * Cin * F + f) * rowlen + j;
    for (int i = 0; i < Cin; ++i) {
        const uint64_t c = src[(int64_t)i * F * rowlen];
#pragma unroll
        for (int k = 0; k < TO; ++k) {
            const int o = o0 + k < Cout ? o0 + k : Cout - 1;
            acc[k] += (uint64_t)w_hat[((int64_t)o * Cin + i) * F + f] * c;
        }
    }
#pragma unroll
    for (int k = 0; k < TO; ++k) {
        const int o = o0 + k;
        if (o >= Cout) break;
        uint64_t v = acc[k];
        if (j == n) v += delta * (uint64_t)r[(b * Cout + o) * F + f];
        ct_out[((b * Cout + o) * F + f) * rowlen + j] = v;
    }
}

static int check_homconv(const ensei_ctx *ctx, const void *ct_in, const void *w, const void *r, int64_t batch,
                         int Cin, int Cout, int64_t F, int n, const void *ct_out, size_t wbytes) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!ct_in || !w || !r || !ct_out || batch <= 0 || Cin <= 0 || Cout <= 0 || F <= 0 || n <= 0)
        return ENSEI_ERR_ARG;
    if (Cin > ENSEI_MAX_CIN || Cout > ENSEI_MAX_COUT || n > ENSEI_MAX_LWE_N || F > (1 << 20)) return ENSEI_ERR_LIMIT;
    if (((uintptr_t)ct_in & 7) || ((uintptr_t)ct_out & 7) || ((uintptr_t)r & 3)) return ENSEI_ERR_ALIGN;
    const size_t inb = (size_t)batch * Cin * F * (n + 1) * 8, outb = (size_t)batch * Cout * F * (n + 1) * 8;
    if (overlaps(ct_out, outb, ct_in, inb) || overlaps(ct_out, outb, w, wbytes) ||
        overlaps(ct_out, outb, r, (size_t)batch * Cout * F * 4))
        return ENSEI_ERR_OVERLAP;
    return ENSEI_OK;
}

}  // namespace ensei

using namespace ensei;

extern "C" {

size_t ensei_wpack_bytes(int Cout, int Cin, int64_t F) {
    if (Cout <= 0 || Cin <= 0 || F <= 0) return 0;
    return (size_t)F * ((Cin + 15) / 16) * ((Cout + 15) / 16 * 16) * 48;
}

int ensei_pack_weights(ensei_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F, int8_t *w_pack,
                       void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!w_hat || !w_pack || Cout <= 0 || Cin <= 0 || F <= 0) return ENSEI_ERR_ARG;
    if (Cin > ENSEI_MAX_CIN || Cout > ENSEI_MAX_COUT || F > (1 << 20)) return ENSEI_ERR_LIMIT;
    if (((uintptr_t)w_hat & 3) || ((uintptr_t)w_pack & 15)) return ENSEI_ERR_ALIGN;
    if (overlaps(w_pack, ensei_wpack_bytes(Cout, Cin, F), w_hat, (size_t)Cout * Cin * F * 4)) return ENSEI_ERR_OVERLAP;
    const int SC = (Cin + 15) / 16, Cout16 = (Cout + 15) / 16 * 16;
    const int64_t total = F * SC * Cout16;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(pack_weights_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, w_hat, Cout,
                       Cin, F, SC, Cout16, w_pack);
    return launch_status();
}

int ensei_homconv(ensei_ctx *ctx, const uint64_t *ct_in, const int8_t *w_pack, const uint32_t *r, int64_t batch,
                  int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, void *stream) {
    int st = check_homconv(ctx, ct_in, w_pack, r, batch, Cin, Cout, F, n, ct_out, ensei_wpack_bytes(Cout, Cin, F));
    if (st) return st;
    if ((uintptr_t)w_pack & 15) return ENSEI_ERR_ALIGN;
    const int SC = (Cin + 15) / 16, Cout16 = (Cout + 15) / 16 * 16;
    const int RB = Cout <= 16 ? 1 : 2;
    const int n_ot = (Cout + 16 * RB - 1) / (16 * RB);
    const int n_jt = (n + 1 + 63) / 64;
    const int n_ks = (Cin + 63) / 64;
    const int64_t n_tiles = batch * F * n_jt * n_ot;
    // persistent grid: two resident workgroups per CU
    int64_t blocks = (int64_t)ctx->num_cus * 2;
    if (n_tiles < blocks) blocks = n_tiles;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)blocks), blk(256);
    if (RB == 1)
        hipLaunchKernelGGL(homconv_mfma_kernel<1>, grid, blk, 0, s, ct_in, w_pack, r, Cin, Cout, F, n, ctx->delta,
                           ct_out, n_ot, n_jt, SC, Cout16, n_tiles, n_ks);
    else
        hipLaunchKernelGGL(homconv_mfma_kernel<2>, grid, blk, 0, s, ct_in, w_pack, r, Cin, Cout, F, n, ctx->delta,
                           ct_out, n_ot, n_jt, SC, Cout16, n_tiles, n_ks);
    return launch_status();
}

int ensei_homconv_valu(ensei_ctx *ctx, const uint64_t *ct_in, const uint32_t *w_hat, const uint32_t *r,
                       int64_t batch, int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, void *stream) {
    int st = check_homconv(ctx, ct_in, w_hat, r, batch, Cin, Cout, F, n, ct_out, (size_t)Cout * Cin * F * 4);
    if (st) return st;
    if ((uintptr_t)w_hat & 3) return ENSEI_ERR_ALIGN;
    constexpr int TO = 16;
    const int n_ot = (Cout + TO - 1) / TO, n_jb = (n + 1 + 255) / 256;
    const int64_t blocks = batch * F * n_ot * n_jb;
    if (blocks > 0x7fffffff) return ENSEI_ERR_LIMIT;
    hipLaunchKernelGGL(homconv_valu_kernel<TO>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, ct_in,
                       w_hat, r, Cin, Cout, F, n, ctx->delta, ct_out, n_jb, n_ot);
    return launch_status();
}

}  // extern "C"
