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

template <int RB>
__global__ __launch_bounds__(256) void homconv_mfma_kernel(const uint64_t *__restrict__ ct_in,
                                                           const int8_t *__restrict__ w_pack,
                                                           const uint32_t *__restrict__ r, int Cin, int Cout,
                                                           int64_t F, int n, uint64_t delta,
                                                           uint64_t *__restrict__ ct_out, int n_ot, int n_jt, int SC,
                                                           int Cout16) {
    // digit planes k = -2..7 at (k + 2) * kPlaneBytes; planes -2 and -1 stay zero
    __shared__ __attribute__((aligned(16))) uint8_t lds[10 * kPlaneBytes];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, l16 = lane & 15;

    int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int ot = (int)(t % n_ot);
    t /= n_ot;
    const int jt = (int)(t % n_jt);
    t /= n_jt;
    const int64_t f = t % F, b = t / F;
    const int o0 = ot * 16 * RB, j0 = jt * 64;
    const int64_t rowlen = (int64_t)n + 1;

    for (int i = tid; i < 2 * kPlaneBytes / 16; i += 256) reinterpret_cast<uint4 *>(lds)[i] = make_uint4(0, 0, 0, 0);

    v4i acc[8][RB];
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[s][rb] = v4i{0, 0, 0, 0};

    // B operand: lane (column l16, slot g) reads plane s - g, or a zero plane for slot 3.
    const int b_base = (g == 3 ? 1 : 2 - g) * kPlaneBytes;
    const int b_step = g == 3 ? 0 : kPlaneBytes;

    const int jl = j0 + lane;  // column this lane loads
    const bool col_ok = jl <= n;
    const uint64_t *src = ct_in + (b * Cin) * F * rowlen + f * rowlen + jl;
    const int64_t ch_stride = F * rowlen;

    for (int kc0 = 0; kc0 < Cin; kc0 += 64) {
        // ---- HBM -> digit planes in LDS (wave = 16-channel group, lane = column)
        uint32_t lo[16], hi[16];
        const int ch0 = kc0 + wave * 16;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            uint64_t v = 0;
            if (col_ok && ch0 + q < Cin) v = src[(int64_t)(ch0 + q) * ch_stride];
            v += 0x8080808080808080ull;
            lo[q] = (uint32_t)v ^ 0x80808080u;
            hi[q] = (uint32_t)(v >> 32) ^ 0x80808080u;
        }
        uint32_t pl[8][4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            transpose4(lo[4 * d], lo[4 * d + 1], lo[4 * d + 2], lo[4 * d + 3], pl[0][d], pl[1][d], pl[2][d], pl[3][d]);
            transpose4(hi[4 * d], hi[4 * d + 1], hi[4 * d + 2], hi[4 * d + 3], pl[4][d], pl[5][d], pl[6][d], pl[7][d]);
        }
        __syncthreads();  // previous step's MFMA reads are done
#pragma unroll
        for (int k = 0; k < 8; ++k)
            *reinterpret_cast<uint4 *>(lds + (k + 2) * kPlaneBytes + (wave * 64 + lane) * 16) =
                make_uint4(pl[k][0], pl[k][1], pl[k][2], pl[k][3]);
        __syncthreads();

        // ---- MFMA: wave owns columns j0 + 16*wave + [0, 16)
#pragma unroll
        for (int sc = 0; sc < 4; ++sc) {
            const int scg = kc0 / 16 + sc;
            if (scg >= SC) break;
            v4i A[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                A[rb] = v4i{0, 0, 0, 0};
                if (g < 3 && o0 + rb * 16 < Cout16)
                    A[rb] = *reinterpret_cast<const v4i *>(
                        w_pack + ((((int64_t)f * SC + scg) * Cout16 + o0 + rb * 16 + l16) * 3 + g) * 16);
            }
            const uint8_t *bp = lds + b_base + (sc * 64 + wave * 16 + l16) * 16;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const v4i B = *reinterpret_cast<const v4i *>(bp + s * b_step);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    acc[s][rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[rb], B, acc[s][rb], 0, 0, 0);
            }
        }
    }

    // ---- epilogue: lane holds rows 4*g + i (i < 4) of column l16 in each row block
    const int jc = j0 + wave * 16 + l16;
    if (jc > n) return;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = o0 + rb * 16 + 4 * g + i;
            if (o >= Cout) continue;
            const int64_t lo64 = (int64_t)acc[0][rb][i] + (int64_t)acc[1][rb][i] * 256 +
                                 (int64_t)acc[2][rb][i] * 65536 + (int64_t)acc[3][rb][i] * 16777216;
            const uint32_t hi32 = (uint32_t)acc[4][rb][i] + ((uint32_t)acc[5][rb][i] << 8) +
                                  ((uint32_t)acc[6][rb][i] << 16) + ((uint32_t)acc[7][rb][i] << 24);
            uint64_t v = (uint64_t)lo64 + ((uint64_t)hi32 << 32);
            if (jc == n) v += delta * (uint64_t)r[(b * Cout + o) * F + f];
            ct_out[((b * Cout + o) * F + f) * rowlen + jc] = v;
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
    const int64_t blocks = batch * F * n_jt * n_ot;
    if (blocks > 0x7fffffff) return ENSEI_ERR_LIMIT;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)blocks), blk(256);
    if (RB == 1)
        hipLaunchKernelGGL(homconv_mfma_kernel<1>, grid, blk, 0, s, ct_in, w_pack, r, Cin, Cout, F, n, ctx->delta,
                           ct_out, n_ot, n_jt, SC, Cout16);
    else if (RB == 2)
        hipLaunchKernelGGL(homconv_mfma_kernel<2>, grid, blk, 0, s, ct_in, w_pack, r, Cin, Cout, F, n, ctx->delta,
                           ct_out, n_ot, n_jt, SC, Cout16);
    else
        hipLaunchKernelGGL(homconv_mfma_kernel<4>, grid, blk, 0, s, ct_in, w_pack, r, Cin, Cout, F, n, ctx->delta,
                           ct_out, n_ot, n_jt, SC, Cout16);
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
