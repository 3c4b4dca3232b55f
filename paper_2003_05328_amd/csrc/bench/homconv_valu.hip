// The vector-ALU HomConv, the comparison point for the matrix-core kernels of
// the product library. Built into libensei_bench.so, which benchmarks and
// tests load; it uses only the public ABI of libensei.so.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ensei_bench.h"

namespace {

// Vector-ALU HomConv: one thread per word index j of one (b, f), TO
// consecutive rows o in registers; the thread walks the Cin contiguous input
// words of its j, and W^[o][i][f] is uniform across the workgroup (scalar
// loads). Each word-MAC is a 32 x 32 -> 64-bit multiply-add plus a low 32-bit
// multiply for the high half.
template <int TO>
__global__ __launch_bounds__(256) void homconv_valu_kernel(const uint64_t *__restrict__ ct_in,
                                                           const uint32_t *__restrict__ w_hat,
                                                           const uint32_t *__restrict__ r, int Cin, int Cout,
                                                           int64_t F, int n, uint64_t delta,
                                                           uint64_t *__restrict__ ct_out, int n_jb, int n_ot) {
    int64_t t = blockIdx.x;
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
    const uint64_t *src = ct_in + ((b * F + f) * rowlen + j) * Cin;
    for (int i = 0; i < Cin; ++i) {
        const uint64_t c = src[i];
#pragma unroll
        for (int k = 0; k < TO; ++k) {
            const int o = o0 + k < Cout ? o0 + k : Cout - 1;
            acc[k] += (uint64_t)w_hat[((int64_t)o * Cin + i) * F + f] * c;
        }
    }
    uint64_t *dst = ct_out + ((b * F + f) * rowlen + j) * Cout;
#pragma unroll
    for (int k = 0; k < TO; ++k) {
        const int o = o0 + k;
        if (o >= Cout) break;
        uint64_t v = acc[k];
        if (j == n) v += delta * (uint64_t)r[(b * Cout + o) * F + f];
        dst[o] = v;
    }
}

bool overlap(const void *a, size_t an, const void *b, size_t bn) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

}  // namespace

extern "C" int ensei_bench_homconv_valu(const ensei_ctx *ctx, const uint64_t *ct_in, const uint32_t *w_hat,
                                        const uint32_t *r, int64_t batch, int Cin, int Cout, int64_t F, int n,
                                        uint64_t *ct_out, void *stream) {
    if (!ctx || !ct_in || !w_hat || !r || !ct_out) return ENSEI_ERR_ARG;
    if (batch <= 0 || Cin <= 0 || Cout <= 0 || F <= 0 || n <= 0) return ENSEI_ERR_ARG;
    if (Cin > ENSEI_MAX_CIN || Cout > ENSEI_MAX_COUT || n > ENSEI_MAX_LWE_N || F > (1 << 20)) return ENSEI_ERR_LIMIT;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ENSEI_ERR_HIP;
    if (dev != ensei_ctx_device(ctx)) return ENSEI_ERR_DEVICE;
    if (((uintptr_t)ct_in & 7) || ((uintptr_t)ct_out & 7) || ((uintptr_t)r & 3) || ((uintptr_t)w_hat & 3))
        return ENSEI_ERR_ALIGN;
    const size_t inb = (size_t)batch * Cin * F * (n + 1) * 8, outb = (size_t)batch * Cout * F * (n + 1) * 8;
    if (overlap(ct_out, outb, ct_in, inb) || overlap(ct_out, outb, w_hat, (size_t)Cout * Cin * F * 4) ||
        overlap(ct_out, outb, r, (size_t)batch * Cout * F * 4))
        return ENSEI_ERR_OVERLAP;
    constexpr int TO = 16;
    const int n_ot = (Cout + TO - 1) / TO, n_jb = (n + 1 + 255) / 256;
    const int64_t blocks = batch * F * n_ot * n_jb;
    if (blocks > 0x7fffffff) return ENSEI_ERR_LIMIT;
    hipLaunchKernelGGL(homconv_valu_kernel<TO>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, ct_in,
                       w_hat, r, Cin, Cout, F, n, ensei_ctx_delta(ctx), ct_out, n_jb, n_ot);
    return hipGetLastError() == hipSuccess ? ENSEI_OK : ENSEI_ERR_HIP;
}
