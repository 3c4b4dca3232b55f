// Chained rounds of the frequency-domain secure convolution (Fig. 2's later
// rounds): HomRec, the server's plaintext addition of its transformed share to
// the client's ciphertexts (Eq. (homrec), Eq. (dft_convolution0)), and a
// stand-in for the oblivious activation computed in the clear, so that a
// round's output shares can feed the next round on one device.
#include "ensei_internal.hpp"

namespace ensei {

// ct [B][F][n+1][C]: the b word of ciphertext (b, c, f) gains
// Delta * s_hat[b][c][f] mod 2^64. The share is channel-major and the b words
// frequency-major, so each block moves a tile of kHrC channels by kHrF
// frequencies of one image through LDS: it reads the share along f (whole
// 128-byte rows) and updates the b words along c (a wave's 64 words are one
// contiguous 512-byte run of a (b, f) block's word row n). Reading the share
// straight along c would touch one line per lane, and the blocks of
// neighbouring f, spread over the XCDs, would fetch each line once per L2.
// 1024 threads move two elements each per phase, so that a tile's few
// dependent memory steps are overlapped by many waves.
constexpr int kHrC = 64, kHrF = 32, kHrThreads = 1024;
static_assert(kHrC * kHrF % kHrThreads == 0 && kHrThreads % kHrF == 0 && kHrThreads % kHrC == 0, "homrec tile");

__global__ __launch_bounds__(kHrThreads) void homrec_kernel(uint64_t *__restrict__ ct,
                                                            const uint32_t *__restrict__ s_hat, int64_t B, int C,
                                                            int64_t F, int n, uint64_t delta) {
    __shared__ uint32_t tile[kHrC][kHrF + 1];
    const int t = threadIdx.x;
    const int64_t c_tiles = (C + kHrC - 1) / kHrC, f_tiles = (F + kHrF - 1) / kHrF;
    const int64_t tiles = B * c_tiles * f_tiles;
    for (int64_t T = blockIdx.x; T < tiles; T += gridDim.x) {
        const int64_t ft = T % f_tiles, rest = T / f_tiles;
        const int c0 = (int)(rest % c_tiles) * kHrC;
        const int64_t b = rest / c_tiles, f0 = ft * kHrF;
        for (int k = 0; k < kHrC * kHrF / kHrThreads; ++k) {
            const int cl = k * (kHrThreads / kHrF) + t / kHrF, fl = t % kHrF;
            if (c0 + cl < C && f0 + fl < F) tile[cl][fl] = s_hat[(b * C + c0 + cl) * F + f0 + fl];
        }
        __syncthreads();
        for (int k = 0; k < kHrC * kHrF / kHrThreads; ++k) {
            const int cl = t % kHrC, fl = k * (kHrThreads / kHrC) + t / kHrC;
            const int64_t f = f0 + fl;
            if (c0 + cl < C && f < F) ct[((b * F + f) * (n + 1) + n) * C + c0 + cl] += delta * (uint64_t)tile[cl][fl];
        }
        __syncthreads();
    }
}

// s_a_next = f((s_a + s_b) mod p) - s_b_next mod p, f the identity (act 0)
// or the square (act 1); every input a residue < p.
__global__ __launch_bounds__(256) void reshare_kernel(const uint32_t *s_a, const uint32_t *s_b,
                                                      const uint32_t *s_b_next, int64_t count, int act, uint32_t p,
                                                      uint32_t *s_a_next) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t y = reduce_once(s_a[k] + s_b[k], p);
        const uint32_t u = act == 1 ? (uint32_t)((uint64_t)y * y % p) : y;
        s_a_next[k] = reduce_once(u + p - s_b_next[k], p);
    }
}

static int64_t grid_for(int64_t items) {
    const int64_t blocks = (items + 255) / 256;
    return blocks < 65536 ? blocks : 65536;
}

}  // namespace ensei

using namespace ensei;

extern "C" {

int ensei_homrec(ensei_ctx *ctx, uint64_t *ct, const uint32_t *s_hat, int64_t batch, int C, int64_t F, int n,
                 void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!ct || !s_hat || batch <= 0 || C <= 0 || F <= 0 || n <= 0) return ENSEI_ERR_ARG;
    if (n > ENSEI_MAX_LWE_N || C > ENSEI_MAX_COUT) return ENSEI_ERR_LIMIT;
    if (batch > ((int64_t)1 << 40) / C / F) return ENSEI_ERR_LIMIT;  // keeps the byte counts below in range
    if (((uintptr_t)ct & 7) || ((uintptr_t)s_hat & 3)) return ENSEI_ERR_ALIGN;
    const size_t num = (size_t)batch * C * F;
    if (overlaps(ct, num * (size_t)(n + 1) * 8, s_hat, num * 4)) return ENSEI_ERR_OVERLAP;
    const int64_t tiles = batch * ((C + kHrC - 1) / kHrC) * ((F + kHrF - 1) / kHrF);
    hipLaunchKernelGGL(homrec_kernel, dim3((unsigned)(tiles < 65536 ? tiles : 65536)), dim3(kHrThreads), 0,
                       (hipStream_t)stream, ct, s_hat, batch, C, F, n, ctx->delta);
    return launch_status();
}

int ensei_homrec_seeded(ensei_ctx *ctx, uint64_t *b_words, const uint32_t *s_hat, int64_t batch, int C, int64_t F,
                        void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!b_words || !s_hat || batch <= 0 || C <= 0 || F <= 0) return ENSEI_ERR_ARG;
    if (C > ENSEI_MAX_COUT || batch > ((int64_t)1 << 40) / C / F) return ENSEI_ERR_LIMIT;
    if (((uintptr_t)b_words & 7) || ((uintptr_t)s_hat & 3)) return ENSEI_ERR_ALIGN;
    const size_t num = (size_t)batch * C * F;
    if (overlaps(b_words, num * 8, s_hat, num * 4)) return ENSEI_ERR_OVERLAP;
    // the compact b words are the word-major layout with no a-words (word n = 0)
    const int64_t tiles = batch * ((C + kHrC - 1) / kHrC) * ((F + kHrF - 1) / kHrF);
    hipLaunchKernelGGL(homrec_kernel, dim3((unsigned)(tiles < 65536 ? tiles : 65536)), dim3(kHrThreads), 0,
                       (hipStream_t)stream, b_words, s_hat, batch, C, F, 0, ctx->delta);
    return launch_status();
}

int ensei_reshare(ensei_ctx *ctx, const uint32_t *s_a, const uint32_t *s_b, const uint32_t *s_b_next, int64_t count,
                  int act, uint32_t *s_a_next, void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!s_a || !s_b || !s_b_next || !s_a_next || count <= 0 || (act != 0 && act != 1)) return ENSEI_ERR_ARG;
    if (((uintptr_t)s_a & 3) || ((uintptr_t)s_b & 3) || ((uintptr_t)s_b_next & 3) || ((uintptr_t)s_a_next & 3))
        return ENSEI_ERR_ALIGN;
    hipLaunchKernelGGL(reshare_kernel, dim3((unsigned)grid_for(count)), dim3(256), 0, (hipStream_t)stream, s_a, s_b,
                       s_b_next, count, act, ctx->p, s_a_next);
    return launch_status();
}

}  // extern "C"
