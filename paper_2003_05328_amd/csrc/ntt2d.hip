// Cyclic 2D NTT / INTT over Z_p for H x W grids (H, W powers of two <= 128),
// the server's share INTT2D(-r), and the filter weight prep (padding fused into the NTT2D's staging).
//
// Layout: one workgroup transforms T whole channels. The channels are staged
// from HBM into LDS with 16-byte loads (rows padded to W+1 words so that
// both row and column accesses are bank-conflict free). Every row is then
// transformed by two threads: the first radix-2 decimation-in-frequency stage
// splits a length-L line into two independent length-L/2 lines (the sums,
// whose transform gives the even outputs, and the twiddled differences, which
// give the odd ones), so thread h = 0 / 1 computes its half of that stage
// from the line in LDS and the rest of its half-length transform in registers
// (fully unrolled, twiddles as uniform scalars), writing outputs 2k + h back
// in natural order. After a barrier the columns are done the same way, the
// inverse's (HW)^-1 applied, and stored straight to HBM with lanes covering
// consecutive columns so the stores coalesce. h is uniform per wave whenever
// a half-phase spans whole waves. HBM traffic is the algorithmic 4 B read +
// 4 B written per point.
#include "ensei_internal.hpp"

namespace ensei {

template <int L>
struct BitRev {
    static constexpr int apply(int k) {
        int r = 0;
        for (int b = 1; b < L; b <<= 1) {
            r = (r << 1) | (k & 1);
            k >>= 1;
        }
        return r;
    }
};

// In-register radix-2 DIF transform of length L. Input residues < 2p in
// natural order; output residues < 2p in bit-reversed order.
// tw: this direction's table; entry (m/2 - 1) + j holds omega_m^j.
template <int L>
__device__ __forceinline__ void dif_line(uint32_t (&v)[L], const uint2 *__restrict__ tw, uint32_t p) {
    const uint32_t p2 = 2 * p;
#pragma unroll
    for (int m = L; m >= 2; m >>= 1) {
        const int h = m >> 1;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            uint2 w = make_uint2(1, 0);
            if (j > 0) w = tw[h - 1 + j];
#pragma unroll
            for (int b = 0; b < L; b += m) {
                const uint32_t u = v[b + j], t = v[b + j + h];
                const uint32_t s = reduce_once(u + t, p2);
                uint32_t d = u - t + p2;  // (0, 4p)
                d = (j == 0) ? reduce_once(d, p2) : mulmod_lazy(d, w.x, w.y, p);
                v[b + j] = s;
                v[b + j + h] = d;
            }
        }
    }
}

// The same transform for p < 2^17 without the per-stage reductions: the
// sums are kept as they are and the differences are offset by the stage's
// input bound B (inputs < B give sums and offset differences < 2 B); a
// twiddle multiplication brings its value back below 2p. From inputs < 2p
// the outputs stay below 2p L <= 128 p < 2^24, the range of the 24-bit
// multiplies, for L <= 64.
template <int L>
__device__ __forceinline__ void dif_line_lazy(uint32_t (&v)[L], const uint2 *__restrict__ tw, uint32_t p) {
    uint32_t B = 2 * p;  // bound of this stage's inputs
#pragma unroll
    for (int m = L; m >= 2; m >>= 1) {
        const int h = m >> 1;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            uint2 w = make_uint2(1, 0);
            if (j > 0) w = tw[h - 1 + j];
#pragma unroll
            for (int b = 0; b < L; b += m) {
                const uint32_t u = v[b + j], t = v[b + j + h];
                const uint32_t d = u - t + B;
                v[b + j] = u + t;
                v[b + j + h] = (j == 0) ? d : mulmod_lazy_su(d, w.x, w.y, p);
            }
        }
        B *= 2;
    }
}

// Half h of a length-L DIF transform of the line x[0], x[st], ..., x[(L-1) st]
// (residues < 2p): the first stage's sums (h = 0) or twiddled differences
// (h = 1), then the length-L/2 transform. out[k] is output 2k + h in
// bit-reversed order of k (residues < 2p).
template <int L>
__device__ __forceinline__ void dif_half(const uint32_t *x, int st, int h, uint32_t (&v)[L / 2],
                                         const uint2 *__restrict__ tw, uint32_t p) {
    constexpr int H2 = L / 2;
    const uint32_t p2 = 2 * p;
    if (h == 0) {
#pragma unroll
        for (int j = 0; j < H2; ++j) v[j] = reduce_once(x[j * st] + x[(j + H2) * st], p2);
    } else {
#pragma unroll
        for (int j = 0; j < H2; ++j) {
            const uint32_t d = x[j * st] - x[(j + H2) * st] + p2;  // (0, 4p)
            if (j == 0) {
                v[j] = reduce_once(d, p2);
            } else {
                const uint2 w = tw[H2 - 1 + j];
                v[j] = mulmod_lazy(d, w.x, w.y, p);
            }
        }
    }
    if constexpr (H2 >= 2) dif_line<H2>(v, tw, p);
}

template <int LOGH, int LOGW>
struct NttShape {
    static constexpr int H = 1 << LOGH, W = 1 << LOGW, F = H * W;
    static constexpr int LMAX = H > W ? H : W;
    static constexpr int T = 2 * LMAX >= 256 ? 1 : 256 / (2 * LMAX);  // channels per workgroup
    static constexpr int NT = 2 * T * LMAX;                           // threads: two per row / column
    static constexpr int STRIDE = W + 1;                               // padded LDS row
    static constexpr int LDS_WORDS = T * H * STRIDE;
};

// MODE 0: forward. MODE 1: inverse, output times `scale` (= (HW)^-1 for
// INTT2D, -(HW)^-1 for the server share). MODE 2: forward transform of
// filters wsrc [batch][kh][kw] (int32), reduced mod p and zero-padded into
// the top-left of the grid while being staged into LDS.
template <int LOGH, int LOGW, int MODE>
__global__ __launch_bounds__((NttShape<LOGH, LOGW>::NT)) void ntt2d_kernel(const uint32_t *in, uint32_t *out,
                                                                         int64_t batch, const uint2 *__restrict__ tw,
                                                                         uint32_t p, uint32_t scale, uint32_t scale_q,
                                                                         const int32_t *__restrict__ wsrc, int kh,
                                                                         int kw) {
    using S = NttShape<LOGH, LOGW>;
    constexpr int H = S::H, W = S::W, F = S::F, T = S::T, NT = S::NT, STR = S::STRIDE;
    extern __shared__ uint32_t lds[];

    const int tid = threadIdx.x;
    const int64_t first = (int64_t)blockIdx.x * T;
    const int nt = (int)((batch - first) < T ? (batch - first) : T);
    const uint32_t *src = in + first * F;

    if constexpr (MODE == 2) {
        // filters: every grid point written once, the taps reduced mod p
        for (int e = tid; e < T * F; e += NT) {
            const int ch = e / F, f = e % F, r = f / W, c = f % W;
            uint32_t v = 0;
            if (ch < nt && r < kh && c < kw) {
                const int32_t x = wsrc[((first + ch) * kh + r) * kw + c] % (int32_t)p;
                v = (uint32_t)(x < 0 ? x + (int32_t)p : x);
            }
            lds[(ch * H + r) * STR + c] = v;
        }
    }
    // HBM -> LDS, 16-byte loads (channels are 16-byte aligned since F >= 4).
    constexpr int VEC = W >= 4 ? 4 : W;
    for (int e = tid * VEC; MODE != 2 && e < T * F; e += NT * VEC) {
        const int row = e / W, col = e % W;
        if (e < nt * F) {
            if constexpr (VEC == 4) {
                const uint4 q = *reinterpret_cast<const uint4 *>(src + e);
                uint32_t *d = lds + row * STR + col;
                d[0] = q.x;
                d[1] = q.y;
                d[2] = q.z;
                d[3] = q.w;
            } else {
                const uint2 q = *reinterpret_cast<const uint2 *>(src + e);
                lds[row * STR + col] = q.x;
                lds[row * STR + col + 1] = q.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < VEC; ++k) lds[row * STR + col + k] = 0;
        }
    }
    __syncthreads();

    const uint2 *twd = tw + (MODE == 1 ? kTwPerDir : 0);
    {  // rows: half h of row tid % (T H); every thread meets the same barriers
        const bool active = tid < 2 * T * H;
        const int h = tid / (T * H), row = tid % (T * H);
        uint32_t v[W / 2];
        uint32_t *rowp = lds + row * STR;  // channel row / H, row row % H
        if (active) dif_half<W>(rowp, 1, h, v, twd, p);
        __syncthreads();  // both halves have read their row before it is overwritten
        if (active) {
#pragma unroll
            for (int k = 0; k < W / 2; ++k) rowp[2 * k + h] = v[BitRev<W / 2>::apply(k)];
        }
        __syncthreads();
    }

    if (tid < 2 * T * W) {  // columns: half h of column tid % (T W)
        const int h = tid / (T * W), cc = tid % (T * W);
        const int ch = cc / W, c = cc % W;
        uint32_t v[H / 2];
        dif_half<H>(lds + ch * H * STR + c, STR, h, v, twd, p);
        if (ch < nt) {
            uint32_t *dst = out + (first + ch) * F + c;
#pragma unroll
            for (int k = 0; k < H / 2; ++k) {
                uint32_t x = v[BitRev<H / 2>::apply(k)];
                if (MODE == 1) x = mulmod_lazy(x, scale, scale_q, p);
                dst[(2 * k + h) * W] = reduce_once(x, p);
            }
        }
    }
}

// Square grids up to 64 x 64 (the image and filter transforms of every
// workload here): one wave transforms G = 64 / L grids at a time with no
// workgroup barrier at all. Lane (g, r) holds row r of grid g in registers
// (16-byte loads straight from HBM), transforms it there (length-L DIF,
// outputs in bit-reversed register order) and writes it to the wave's own LDS
// tile (rows padded to L + 1 words: conflict-free both ways); lane (g, c) then
// reads column c, transforms it in registers, and stores output row k of all
// the wave's columns with one coalesced store per k. Per point this is one
// LDS write and one read, and every butterfly is in registers. The waves are
// persistent: while a wave works on one group of grids, the rows of its next
// group are already on their way into registers, so the HBM latency hides
// behind the butterflies (the LDS tiles, not the registers, bound the waves
// per CU, so the prefetch costs no occupancy).
// MODE as for ntt2d_kernel; wsrc/kh/kw for MODE 2. LAZY (p < 2^17): the
// line transforms skip their per-stage reductions (dif_line_lazy); one
// Barrett step (reduce_2p, pm = floor(2^32 / p)) brings the rows back below
// 2p before the columns, and the outputs before the final reduction.
constexpr int kNttWaves = 4;  // waves per workgroup

template <int LOGL, int MODE, bool LAZY>
__global__ __launch_bounds__(kNttWaves * 64) void ntt2d_wave_kernel(const uint32_t *in, uint32_t *out, int64_t batch,
                                                                   const uint2 *__restrict__ tw, uint32_t p,
                                                                   uint32_t scale, uint32_t scale_q,
                                                                   const int32_t *__restrict__ wsrc, int kh, int kw,
                                                                   uint32_t pm) {
    constexpr int L = 1 << LOGL, F = L * L, G = 64 / L, STR = L + 1;
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *tile = lds + wave * (G * L * STR);
    const int g = lane / L, i = lane % L;  // rows phase: row i of grid g; columns phase: column i
    const uint2 *twd = tw + (MODE == 1 ? kTwPerDir : 0);
    const int64_t units = (batch + G - 1) / G, stride = (int64_t)gridDim.x * kNttWaves;

    // row i of grid g of unit u into nxt (zero past the batch)
    uint32_t nxt[L];
    auto load_rows = [&](int64_t u) {
        const int64_t grid = u * G + g;
        const bool live = grid < batch;
        if (MODE == 2) {
#pragma unroll
            for (int k = 0; k < L; ++k) {
                uint32_t x = 0;
                if (live && i < kh && k < kw) {
                    const int32_t t = wsrc[(grid * kh + i) * kw + k] % (int32_t)p;
                    x = (uint32_t)(t < 0 ? t + (int32_t)p : t);
                }
                nxt[k] = x;
            }
        } else if constexpr (L >= 4) {
            const uint4 *src = reinterpret_cast<const uint4 *>(in + grid * F + i * L);
#pragma unroll
            for (int q = 0; q < L / 4; ++q) {
                const uint4 x = live ? src[q] : make_uint4(0, 0, 0, 0);
                nxt[4 * q] = x.x;
                nxt[4 * q + 1] = x.y;
                nxt[4 * q + 2] = x.z;
                nxt[4 * q + 3] = x.w;
            }
        } else {
            const uint2 x = live ? *reinterpret_cast<const uint2 *>(in + grid * F + i * L) : make_uint2(0, 0);
            nxt[0] = x.x;
            nxt[1] = x.y;
        }
    };

    int64_t u = (int64_t)blockIdx.x * kNttWaves + wave;
    if (u < units) load_rows(u);
    for (; u < units; u += stride) {
        uint32_t v[L];
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = nxt[k];
        // the next group's rows, in flight during this group's transforms
        if (u + stride < units) load_rows(u + stride);
        // rows
        if (LAZY) {
            dif_line_lazy<L>(v, twd, p);
#pragma unroll
            for (int k = 0; k < L; ++k) v[k] = reduce_2p(v[k], pm, p);
        } else {
            dif_line<L>(v, twd, p);
        }
        uint32_t *row = tile + (g * L + i) * STR;
#pragma unroll
        for (int k = 0; k < L; ++k) row[k] = v[BitRev<L>::apply(k)];
        // the tile is the wave's own: lanes only need each other's writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // columns
        const uint32_t *col = tile + g * L * STR + i;
#pragma unroll
        for (int r = 0; r < L; ++r) v[r] = col[r * STR];
        // every lane has read its column before the next group's rows are written
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (LAZY)
            dif_line_lazy<L>(v, twd, p);
        else
            dif_line<L>(v, twd, p);
        const int64_t grid = u * G + g;
        if (grid < batch) {
            uint32_t *dst = out + grid * F + i;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                uint32_t x = v[BitRev<L>::apply(k)];
                if (MODE == 1)
                    x = mulmod_lazy(x, scale, scale_q, p);
                else if (LAZY)
                    x = reduce_2p(x, pm, p);
                dst[k * L] = reduce_once(x, p);
            }
        }
    }
}

template <int LOGH, int LOGW, int MODE>
static int launch_ntt(const uint32_t *in, uint32_t *out, int64_t batch, const ensei_ctx *ctx, uint32_t scale,
                      hipStream_t st, const int32_t *w, int kh, int kw) {
    const uint32_t scale_q = (uint32_t)(((uint64_t)scale << 24) / ctx->p);
    if constexpr (LOGH == LOGW && LOGH <= 6) {
        constexpr int L = 1 << LOGH, G = 64 / L;
        const size_t lds = (size_t)kNttWaves * G * L * (L + 1) * 4;
        const bool lazy = ctx->p < (1u << 17);
        auto kern = lazy ? ntt2d_wave_kernel<LOGH, MODE, true> : ntt2d_wave_kernel<LOGH, MODE, false>;
        static std::atomic<bool> wave_attr[kMaxDevices][2];  // dynamic-LDS limit raised, by device and form
        const bool cached = ctx->device < kMaxDevices;
        if (lds > 48 * 1024 && (!cached || !wave_attr[ctx->device][lazy].load(std::memory_order_acquire))) {
            if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
                hipSuccess)
                return ENSEI_ERR_HIP;
            if (cached) wave_attr[ctx->device][lazy].store(true, std::memory_order_release);
        }
        // persistent: as many workgroups as are resident at once, none idle
        static std::atomic<int> resident[kMaxDevices][2];  // workgroups per CU (0: not yet known), by device and form
        int per_cu = cached ? resident[ctx->device][lazy].load(std::memory_order_relaxed) : 0;
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNttWaves * 64, lds) != hipSuccess ||
                per_cu < 1)
                per_cu = 1;
            if (cached) resident[ctx->device][lazy].store(per_cu, std::memory_order_relaxed);
        }
        const int64_t needed = (batch + kNttWaves * G - 1) / (kNttWaves * G);
        const int64_t full = (int64_t)ctx->num_cus * per_cu;
        const int64_t blocks = needed < full ? needed : full;
        const uint32_t pm = (uint32_t)((1ull << 32) / ctx->p);
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNttWaves * 64), lds, st, in, out, batch, ctx->d_tw,
                           ctx->p, scale, scale_q, w, kh, kw, pm);
        return launch_status();
    }
    using S = NttShape<LOGH, LOGW>;
    const size_t lds = (size_t)S::LDS_WORDS * 4;
    auto kern = ntt2d_kernel<LOGH, LOGW, MODE>;
    static std::atomic<bool> attr_set[kMaxDevices];  // dynamic-LDS limit raised, by device
    const bool cached = ctx->device < kMaxDevices;
    if (lds > 48 * 1024 && (!cached || !attr_set[ctx->device].load(std::memory_order_acquire))) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return ENSEI_ERR_HIP;
        if (cached) attr_set[ctx->device].store(true, std::memory_order_release);
    }
    const int64_t blocks = (batch + S::T - 1) / S::T;
    if (blocks > 0x7fffffff) return ENSEI_ERR_LIMIT;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(S::NT), lds, st, in, out, batch, ctx->d_tw, ctx->p, scale,
                       scale_q, w, kh, kw);
    return launch_status();
}

using LaunchFn = int (*)(const uint32_t *, uint32_t *, int64_t, const ensei_ctx *, uint32_t, hipStream_t,
                        const int32_t *, int, int);

template <int MODE>
struct NttTable {
    template <int LH, int LW>
    static constexpr LaunchFn entry() {
        return &launch_ntt<LH, LW, MODE>;
    }
#define ENSEI_ROW(LH) \
    entry<LH, 1>(), entry<LH, 2>(), entry<LH, 3>(), entry<LH, 4>(), entry<LH, 5>(), entry<LH, 6>(), entry<LH, 7>()
    static constexpr LaunchFn table[7][7] = {{ENSEI_ROW(1)}, {ENSEI_ROW(2)}, {ENSEI_ROW(3)}, {ENSEI_ROW(4)},
                                             {ENSEI_ROW(5)}, {ENSEI_ROW(6)}, {ENSEI_ROW(7)}};
#undef ENSEI_ROW
};

static uint64_t host_powmod32(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    for (; e; e >>= 1) {
        if (e & 1) r = r * a % p;
        a = a * a % p;
    }
    return r;
}

// Validates a transform call; on success fills lh, lw.
static int check_ntt(const ensei_ctx *ctx, const void *in, const void *out, int64_t batch, int H, int W, int *lh,
                     int *lw) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!in || !out || batch <= 0) return ENSEI_ERR_ARG;
    *lh = ilog2_pow2(H);
    *lw = ilog2_pow2(W);
    if (*lh < 1 || *lw < 1 || *lh > ctx->max_log || *lw > ctx->max_log) return ENSEI_ERR_SHAPE;
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return ENSEI_ERR_ALIGN;
    const size_t bytes = (size_t)batch * H * W * 4;
    if (in != out && overlaps(in, bytes, out, bytes)) return ENSEI_ERR_OVERLAP;
    return ENSEI_OK;
}

static int run_ntt(const ensei_ctx *ctx, const uint32_t *in, uint32_t *out, int64_t batch, int H, int W, int mode,
                   bool negate, void *stream) {
    int lh, lw;
    int st = check_ntt(ctx, in, out, batch, H, W, &lh, &lw);
    if (st) return st;
    uint32_t scale = 1;
    if (mode == 1) {
        scale = (uint32_t)host_powmod32((uint64_t)H * W % ctx->p, ctx->p - 2, ctx->p);
        if (negate) scale = (ctx->p - scale) % ctx->p;
    }
    LaunchFn fn = mode == 0 ? NttTable<0>::table[lh - 1][lw - 1] : NttTable<1>::table[lh - 1][lw - 1];
    return fn(in, out, batch, ctx, scale, (hipStream_t)stream, nullptr, 0, 0);
}

}  // namespace ensei

using namespace ensei;

extern "C" {

int ensei_ntt2d(ensei_ctx *ctx, const uint32_t *in, uint32_t *out, int64_t batch, int H, int W, void *stream) {
    return run_ntt(ctx, in, out, batch, H, W, 0, false, stream);
}

int ensei_intt2d(ensei_ctx *ctx, const uint32_t *in, uint32_t *out, int64_t batch, int H, int W, void *stream) {
    return run_ntt(ctx, in, out, batch, H, W, 1, false, stream);
}

int ensei_server_share(ensei_ctx *ctx, const uint32_t *r, uint32_t *s_b, int64_t batch, int H, int W,
                       void *stream) {
    return run_ntt(ctx, r, s_b, batch, H, W, 1, true, stream);
}

int ensei_weight_prep(ensei_ctx *ctx, const int32_t *w, int Cout, int Cin, int kh, int kw, int H, int W,
                      uint32_t *w_hat, void *stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!w || !w_hat || Cout <= 0 || Cin <= 0 || kh <= 0 || kw <= 0) return ENSEI_ERR_ARG;
    int lh = ilog2_pow2(H), lw = ilog2_pow2(W);
    if (lh < 1 || lw < 1 || lh > ctx->max_log || lw > ctx->max_log) return ENSEI_ERR_SHAPE;
    if (kh > H || kw > W) return ENSEI_ERR_SHAPE;
    if (((uintptr_t)w & 3) || ((uintptr_t)w_hat & 15)) return ENSEI_ERR_ALIGN;
    const int64_t nfilt = (int64_t)Cout * Cin;
    if (overlaps(w, (size_t)nfilt * kh * kw * 4, w_hat, (size_t)nfilt * H * W * 4)) return ENSEI_ERR_OVERLAP;
    // one pass: taps reduced and padded while staged into LDS, then the forward transform
    return NttTable<2>::table[lh - 1][lw - 1](nullptr, w_hat, nfilt, ctx, 1, (hipStream_t)stream, w, kh, kw);
}

}  // extern "C"
