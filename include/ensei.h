/*
 * ensei.h — C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of ENSEI's frequency-domain secure convolution (Bian et al., "ENSEI:
 * Efficient Secure Inference via Frequency-Domain Homomorphic Convolution for
 * Privacy-Preserving Visual Recognition", CVPR 2020).
 *
 * One secure convolution (the start round of the protocol in Fig. 2) is,
 * with p one prime used as NTT, share and plaintext modulus and q = 2^64 the
 * ciphertext modulus:
 *   client:  x^ = NTT2D(x)                 ensei_ntt2d      (client transforms its input)
 *            ct_in = Enc(x^, s)            ensei_encrypt    (and encrypts it)
 *   server:  W^ = NTT2D(pad(w))            ensei_weight_prep + ensei_pack_weights (setup)
 *            ct_out = sum_i W^ ct_in + Delta r   ensei_homconv (Hadamard product, HomShare)
 *   client:  m = Dec(ct_out, s)            ensei_decrypt    (client decrypts)
 *            s_A = INTT2D(m)               ensei_intt2d     (both parties take the inverse
 *   server:  s_B = INTT2D(-r)              ensei_server_share  transform of their shares)
 * and s_A + s_B = x (*) w mod p (Sec. 4.1, Appendix A).
 *
 * Beyond that round: later rounds chain through ensei_reshare (a stand-in for
 * the activation, in the clear) and ensei_homrec (the server adds its share
 * to the client's fresh ciphertexts); seeded ciphertexts keep only their b
 * words (ensei_encrypt_seeded, ensei_homconv_seeded, ensei_plan_create_seeded);
 * ensei_sample_errors draws Enc's errors on the device; batched plans and a
 * serving layer run many convolutions.
 *
 * Common rules for every call below:
 *   - every array pointer is a DEVICE pointer on the context's device (the
 *     calls that take host memory say so), owned by the caller, who keeps it alive until the work queued on `stream`
 *     has finished; the library never frees, retains or allocates on a call;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     every call only enqueues work on it and returns without synchronising;
 *   - arrays are dense, row-major, with the shapes stated per call;
 *   - argument checks run on the host before any launch; a call that returns
 *     an error has enqueued nothing. Errors raised later by the device are
 *     not reported by these calls (a HIP launch failure is, as ENSEI_ERR_HIP);
 *   - the current HIP device must be the context's device (ENSEI_ERR_DEVICE);
 *   - unless stated, outputs must not overlap inputs (ENSEI_ERR_OVERLAP).
 */
#ifndef ENSEI_H
#define ENSEI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ensei_status {
    ENSEI_OK = 0,
    ENSEI_ERR_ARG = -1,     /* null pointer, non-positive size, bad flag */
    ENSEI_ERR_SHAPE = -2,   /* H or W not a power of two in [2, 128], or not dividing p-1 */
    ENSEI_ERR_MODULUS = -3, /* p not prime, or outside [3, 2^22) */
    ENSEI_ERR_ALIGN = -4,   /* pointer not aligned to its element size */
    ENSEI_ERR_OVERLAP = -5, /* output range overlaps an input range */
    ENSEI_ERR_LIMIT = -6,   /* size beyond the supported range (see each call) */
    ENSEI_ERR_DEVICE = -7,  /* current HIP device is not the context's device */
    ENSEI_ERR_HIP = -8,     /* HIP runtime error (allocation at create, launch failure) */
    ENSEI_ERR_TIMEOUT = -9, /* a wait ended before the request finished (serving) */
    ENSEI_ERR_BUDGET = -10, /* a request does not fit the server's budget or queue limit (serving) */
    ENSEI_ERR_CANCELLED = -11, /* the request was cancelled (serving) */
    ENSEI_ERR_STATE = -12   /* the request has already finished (serving) */
};

/* Largest supported sizes. */
#define ENSEI_MAX_DIM 128        /* H and W */
#define ENSEI_MAX_LWE_N 16384    /* LWE dimension n */
#define ENSEI_MAX_CIN 32768      /* input channels of HomConv (keeps i32 limb sums exact) */
#define ENSEI_MAX_COUT 65536     /* output channels of HomConv */

typedef struct ensei_ctx ensei_ctx;

/* Creates a context for prime modulus p on HIP device `device`: checks that
 * p is prime with 3 <= p < 2^22 (the bound keeps every lazily reduced residue
 * below 2^24, the width of the 24-bit multipliers the transforms use), finds
 * the smallest primitive root g, and uploads the twiddle tables
 * omega_L^j = g^((p-1)/L * j) for every power-of-two L <= 128 dividing p-1
 * (Eq. (ntt_transform_eq)). Delta = floor(2^64 / p) (Eq. (bfv_enc), q = 2^64).
 * Allocates a few KB of device memory; this is the only allocating call.
 * On error *out is set to NULL. */
int ensei_ctx_create(ensei_ctx **out, uint32_t p, int device);

/* Frees the context (NULL is a no-op). The caller must have finished all
 * work that uses it. */
int ensei_ctx_destroy(ensei_ctx *ctx);

/* Static human-readable text for a status code. */
const char *ensei_status_str(int status);

/* The context's p, Delta = floor(2^64/p), largest usable transform size and
 * HIP device (-1 for a NULL context). */
int ensei_ctx_device(const ensei_ctx *ctx);
uint32_t ensei_ctx_modulus(const ensei_ctx *ctx);
uint64_t ensei_ctx_delta(const ensei_ctx *ctx);
int ensei_ctx_max_dim(const ensei_ctx *ctx);

/* ----------------------------------------------------------- transforms --
 * Cyclic 2D NTT over Z_p of `batch` channels, each an H x W grid
 * (Sec. 4.1, "Line 1-3": 2D DFT of the padded input; Eq. (ntt_transform_eq)
 * along both axes):
 *   out[t][k1*W + k2] = sum_{i1<H, i2<W} in[t][i1*W + i2]
 *                       * omega_H^(i1*k1) * omega_W^(i2*k2)  mod p,
 * with omega_N = g^((p-1)/N). in: uint32 [batch][H][W], every value < p;
 * out: uint32 [batch][H*W], flattened row-major (f = k1*W + k2), values in
 * [0, p). H, W: powers of two in [2, min(128, ctx max dim)].
 * In-place (in == out) is allowed; other overlap is not. */
int ensei_ntt2d(ensei_ctx *ctx, const uint32_t *in, uint32_t *out, int64_t batch, int H, int W,
                void *stream);

/* The inverse (Sec. 4.1, "Line 4-6"): omega^-1 and a final factor (H W)^-1:
 *   out[t][i1][i2] = (HW)^-1 sum_{k1,k2} in[t][k1*W + k2]
 *                    * omega_H^(-i1*k1) * omega_W^(-i2*k2)  mod p.
 * Same layouts and rules as ensei_ntt2d (in: [batch][H*W] values < p;
 * out: [batch][H][W]). */
int ensei_intt2d(ensei_ctx *ctx, const uint32_t *in, uint32_t *out, int64_t batch, int H, int W,
                 void *stream);

/* The server's spatial share s_B = INTT2D(-r mod p) of HomShare
 * (Eq. (homshare); Sec. 4.1, "Line 4-6"), for masks r: uint32 [batch][H*W]
 * with values < p; s_b: uint32 [batch][H][W]. The client's share
 * s_A = INTT2D(Dec(ct_out)) then satisfies s_A + s_B = x (*) w mod p.
 * In-place allowed. */
int ensei_server_share(ensei_ctx *ctx, const uint32_t *r, uint32_t *s_b, int64_t batch, int H, int W,
                       void *stream);

/* ---------------------------------------------------------- weight prep --
 * Server setup (Sec. 4.1, "Line 3-4"): each filter w[o][i] (kh x kw signed
 * integers) is reduced mod p, zero-padded into the top-left kh x kw corner
 * of the H x W grid, and transformed by NTT2D:
 *   w_hat[o][i][f] = NTT2D(pad(w[o][i] mod p))[f].
 * w: int32 [Cout][Cin][kh][kw]; w_hat: uint32 [Cout][Cin][H*W] in [0, p).
 * 1 <= kh <= H, 1 <= kw <= W. */
int ensei_weight_prep(ensei_ctx *ctx, const int32_t *w, int Cout, int Cin, int kh, int kw, int H, int W,
                      uint32_t *w_hat, void *stream);

/* Bytes of the packed-weight buffer ensei_pack_weights writes:
 * F * ceil(Cin/64) * ceil(Cout/64) * U * 16 with U = 768 when Cin >= 48,
 * else U = 256 * ceil(Cin/16). Returns 0 for invalid sizes. */
size_t ensei_wpack_bytes(int Cout, int Cin, int64_t F);

/* Packs transformed weights for ensei_homconv: every W^[o][i][f] (the
 * integer in [0, p), p < 2^22) is written as three signed bytes
 * d0 + 2^8 d1 + 2^16 d2 with d0, d1, d2 in [-128, 127] (balanced base-256
 * digits), arranged as the matrix-core operand fragments ensei_homconv
 * loads: for every frequency f, 64-channel step and 64-row output tile, U
 * 16-byte items (one digit of 16 channels for one output row each; rows and
 * channels past Cout and Cin are zero). The arrangement is private to
 * ensei_homconv; only the size above is part of the interface.
 * w_hat: uint32 [Cout][Cin][F]; w_pack: ensei_wpack_bytes(Cout, Cin, F)
 * bytes, 16-byte aligned. */
int ensei_pack_weights(ensei_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F, int8_t *w_pack,
                       void *stream);

/* ------------------------------------------------- ciphertext storage --
 * LWE ciphertexts (one per frequency coefficient) are stored WORD-MAJOR:
 * for B images, C channels and F frequencies, ct is uint64 [B][F][n+1][C]
 * and ciphertext (b, c, f) keeps its word j (j < n: a_j, j = n: b) at
 * ct[b][f][j][c]. Its ciphertext index is q = (b*F + f)*C + c. For one
 * (b, f) the C ciphertexts form a contiguous (n+1) x C matrix, the operand
 * HomConv contracts; with C = 1 the layout is a plain list of rows [N][n+1].
 * Plaintexts, errors, decryptions and masks use the spectra's channel-major
 * layout [B][C][F] (what ensei_ntt2d produces and ensei_intt2d consumes).
 */

/* ------------------------------------------------------------------ Enc --
 * LWE encryption of the B*C*F plaintexts m[b][c][f] < p under the ternary
 * key s (Eq. (bfv_enc) with one coefficient per ciphertext; q = 2^64):
 *   a_j = SplitMix64 output number (ct_index0 + q)*n + j + 1 of the
 *         generator seeded with seed_a, for j < n (the uniform "encryption
 *         constants" the paper generates offline, Sec. 5.1);
 *   b   = sum_j s_j a_j + e[b][c][f] + Delta * m[b][c][f]  mod 2^64.
 * m: uint32 [B][C][F]; s: int8 [n] in {-1, 0, 1}; e: int32 [B][C][F];
 * ct: uint64 [B][F][n+1][C] (word-major, above; 8-byte aligned).
 * 1 <= n <= ENSEI_MAX_LWE_N. Encrypting a slice with ct_index0 = the index of
 * its first ciphertext reproduces the same words as one call over the whole
 * range (C = 1 slices of a list). */
int ensei_encrypt(ensei_ctx *ctx, const uint32_t *m, const int8_t *s, const int32_t *e, int64_t batch, int C,
                  int64_t F, int n, uint64_t seed_a, uint64_t ct_index0, uint64_t *ct, void *stream);

/* -------------------------------------------------------------- HomConv --
 * Server-side homomorphic convolution in the frequency domain: the
 * homomorphic Hadamard product with the transformed filters, summed over
 * input channels, then HomShare's mask (Fig. 2; HomShare in Sec. 3.2):
 *   ct_out(b, o, f)[j] = sum_i W^[o][i][f] * ct_in(b, i, f)[j]  mod 2^64,  j <= n
 *   ct_out(b, o, f)[n] += Delta * r[b][o][f]                      mod 2^64
 * so Dec(ct_out(b, o, f)) = (sum_i W^ x^ + r) mod p and the server keeps -r.
 * ct_in: uint64 [batch][F][n+1][Cin] (word-major); w_pack: from
 * ensei_pack_weights for (Cout, Cin, F); r: uint32 [batch][Cout][F] (< p);
 * ct_out: uint64 [batch][F][n+1][Cout] (word-major). 1 <= Cin <= ENSEI_MAX_CIN,
 * 1 <= Cout <= ENSEI_MAX_COUT, 1 <= n <= ENSEI_MAX_LWE_N, one (b, f) block
 * of either side below 2^31 bytes ((n+1) * max(Cin, Cout) * 8) and one
 * image's masks below 2^31 bytes (Cout * F * 4), else ENSEI_ERR_LIMIT. Runs on the
 * i8 matrix cores (signed-byte limbs of both operands, exact i32 sums,
 * recombined mod 2^64); the kernel is chosen by shape (narrow inputs, deep
 * layers with several output tiles, or the streaming kernel), the results
 * are the same bits. */
int ensei_homconv(ensei_ctx *ctx, const uint64_t *ct_in, const int8_t *w_pack, const uint32_t *r, int64_t batch,
                  int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, void *stream);

/* ------------------------------------------------------------------ Dec --
 * Decryption with round-half-up (Sec. 3.1, "round off the fractions"):
 *   phi  = b - sum_j s_j a_j  mod 2^64,
 *   m[b][c][f] = floor((phi * p + 2^63) / 2^64) mod p   (exact 81-bit arithmetic)
 * for every ciphertext (b, c, f) of ct: uint64 [B][F][n+1][C] (word-major);
 * s: int8 [n]; m: uint32 [B][C][F]. */
int ensei_decrypt(ensei_ctx *ctx, const uint64_t *ct, const int8_t *s, int64_t batch, int C, int64_t F, int n,
                  uint32_t *m, void *stream);

/* ----------------------------------------------------- chained rounds --
 * HomRec (Eq. (homrec) in Sec. 3.2; Fig. 2's re-entry of the server's share, Eq.
 * (dft_convolution0)): the server adds its transformed share to the client's
 * ciphertexts as a plaintext, [s_A] (+) s_B = [s_A + s_B mod p], so that the
 * next round's HomConv runs on an encryption of the whole activation. In
 * place: the b word of ciphertext (b, c, f) of ct: uint64 [batch][F][n+1][C]
 * (word-major) gains Delta * s_hat[b][c][f] mod 2^64, s_hat: uint32
 * [batch][C][F] with values < p (the server's share, transformed by
 * ensei_ntt2d). Since Delta * p = 2^64 - 1, a sum that wraps past p adds -1
 * to the ciphertext's noise. The a-words are not touched. 1 <= n <=
 * ENSEI_MAX_LWE_N, 1 <= C <= ENSEI_MAX_COUT, batch*C*F <= 2^40 (else
 * ENSEI_ERR_LIMIT); ct 8-byte and s_hat 4-byte aligned and not overlapping. */
int ensei_homrec(ensei_ctx *ctx, uint64_t *ct, const uint32_t *s_hat, int64_t batch, int C, int64_t F, int n,
                 void *stream);

/* HomRec on seeded ciphertexts (ensei_encrypt_seeded): the same addition on
 * the compact b words, b_words: uint64 [batch][F][C] (8-byte aligned), in
 * place; the a-words stay implicit in (seed_a, ct_index0). Limits and errors
 * as ensei_homrec. */
int ensei_homrec_seeded(ensei_ctx *ctx, uint64_t *b_words, const uint32_t *s_hat, int64_t batch, int C, int64_t F,
                        void *stream);

/* A stand-in for the oblivious activation between the rounds of Fig. 2,
 * computed in the clear so that chained rounds can run on one device (the
 * garbled-circuit or triplet evaluation itself is outside this library):
 *   s_a_next[k] = f((s_a[k] + s_b[k]) mod p) - s_b_next[k]  mod p,
 * f the identity (act 0) or the square mod p (act 1), for count residues
 * < p in each array (uint32); s_b_next is the server's fresh share. The
 * output may alias any input. ENSEI_ERR_ARG for another act. */
int ensei_reshare(ensei_ctx *ctx, const uint32_t *s_a, const uint32_t *s_b, const uint32_t *s_b_next, int64_t count,
                  int act, uint32_t *s_a_next, void *stream);

/* Errors for Enc drawn on the device: e[b][c][f] (int32 [B][C][F], 4-byte
 * aligned) from the rounded Gaussian of sigma = 3.2 (the LWE error of Sec.
 * 3.1), one output of the public SplitMix64 generator seeded with seed_e per
 * ciphertext: number ct_index0 + q + 1 for the ciphertext index
 * q = (b*F + f)*C + c of ensei_encrypt. Its top bit is the sign and bits
 * 15..62 a uniform v < 2^48; |e| is the number of thresholds
 * T[k] = floor(2^48 erf((k + 1/2) / (sigma sqrt 2))), k < 32, with T[k] <= v
 * (so |e| <= 32). The context computes the thresholds when it is created.
 * batch*C*F <= 2^40, else ENSEI_ERR_LIMIT. */
int ensei_sample_errors(ensei_ctx *ctx, uint64_t seed_e, uint64_t ct_index0, int64_t batch, int C, int64_t F,
                        int32_t *e, void *stream);

/* The sampler's 32 thresholds, copied to out (host memory, n >= 32 entries);
 * returns 32, or ENSEI_ERR_ARG. */
int ensei_error_table(const ensei_ctx *ctx, uint64_t *out, int n);

/* --------------------------------------------------- seeded ciphertexts --
 * The a-words of every ciphertext are the public stream of Enc above (the
 * encryption constants that Sec. 5.1 generates offline), so a batch of
 * ciphertexts is fully given by (seed_a, ct_index0) and its b words: only the
 * b words need to be stored or sent, and the server regenerates the a-words
 * inside HomConv instead of reading them.
 *
 * Enc that keeps only the b words: b_out: uint64 [B][F][C] with
 * b_out[b][f][c] = word n of ensei_encrypt's ciphertext (b, c, f) for the same
 * arguments (8-byte aligned, not overlapping m, s or e). Limits and errors as
 * ensei_encrypt. */
int ensei_encrypt_seeded(ensei_ctx *ctx, const uint32_t *m, const int8_t *s, const int32_t *e, int64_t batch, int C,
                         int64_t F, int n, uint64_t seed_a, uint64_t ct_index0, uint64_t *b_out, void *stream);

/* HomConv of seeded ciphertexts: the same ct_out, bit for bit, as
 * ensei_homconv on the word-major ciphertexts whose word j < n of ciphertext
 * (b, i, f) is SplitMix64 output number (ct_index0 + q)*n + j + 1 of seed_a
 * (q = (b*F + f)*Cin + i, as ensei_encrypt) and whose word n is
 * b_in[b][f][i]; b_in: uint64 [batch][F][Cin], 8-byte aligned.
 * w_pack, r, ct_out, limits and errors as ensei_homconv; the input side
 * moves 8 bytes per ciphertext instead of 8 (n+1). The kernel is chosen by
 * shape as for ensei_homconv (narrow inputs, deep layers, or the streaming
 * kernel), each in its seeded form. */
int ensei_homconv_seeded(ensei_ctx *ctx, const uint64_t *b_in, uint64_t seed_a, uint64_t ct_index0,
                         const int8_t *w_pack, const uint32_t *r, int64_t batch, int Cin, int Cout, int64_t F, int n,
                         uint64_t *ct_out, void *stream);

/* ------------------------------------------------------ batched plans --
 * A plan runs a stack of independent secure convolutions (Fig. 2's start
 * round for each layer; layers of uneven shapes, each over a batch of images
 * of one client) as one captured HIP graph: per layer NTT2D and Enc, then ONE
 * persistent matrix-core HomConv launch over the tiles of all layers (those
 * with at most 8 input channels, and those with several 64-row output tiles
 * and at most 256 input channels, each run their own HomConv kernel after
 * it), then per layer Dec, INTT2D and the server share. The server's filters
 * are transformed and packed once, when the plan is created.
 *
 * The HomConv tile schedule (persistent workgroups; contiguous tile ranges
 * or chunks of 1..256 tiles dealt round-robin; or no shared launch at all,
 * each of those layers in a launch of its own) is picked by timing the
 * candidates on the plan's own shapes and buffers at creation. With a
 * non-NULL tune_cache path the choice is looked up there first, keyed by the
 * device and the layer shapes, and appended after tuning (a text file, one
 * line "key blocks chunk [us]" per entry; the last matching line wins and a
 * line whose key is "*" matches every plan, which pins a schedule). Tuning
 * and the cache never change results.
 *
 * ensei_layer: shape, the server's filters, and the caller's device buffers.
 * Shapes and layouts are those of the single calls (F = H*W):
 *   w [Cout][Cin][kh][kw] int32 (read at creation only);
 *   per run, read:  x [batch][Cin][H][W] residues < p, s [n] ternary int8,
 *                   e [batch][Cin][F] int32, r [batch][Cout][F] masks < p;
 *   per run, written: x_hat [batch][Cin][F], ct_in [batch][F][n+1][Cin],
 *                   ct_out [batch][F][n+1][Cout], m [batch][Cout][F],
 *                   s_a and s_b [batch][Cout][H][W] (client and server shares).
 * The plan keeps the pointers: the buffers must stay valid and unmoved until
 * ensei_plan_destroy, and runs see their current contents. Word j of
 * ciphertext (b, c, f) of layer l is keyed by seed_a of layer l and
 * q = (b*F + f)*Cin + c, exactly as ensei_encrypt with ct_index0 = 0. */
typedef struct ensei_plan ensei_plan;

typedef struct ensei_layer {
    int H, W, Cin, Cout, kh, kw, n;
    int64_t batch;
    uint64_t seed_a;
    const int32_t *w;
    const uint32_t *x;
    const int8_t *s;
    const int32_t *e;
    const uint32_t *r;
    uint32_t *x_hat;
    uint64_t *ct_in;
    uint64_t *ct_out;
    uint32_t *m;
    uint32_t *s_a;
    uint32_t *s_b;
} ensei_layer;

/* The HomConv schedule a plan runs: persistent workgroups, chunk (0 =
 * contiguous tile ranges, -1 = a launch per layer instead of the shared
 * one), the measured time of its HomConv launches in
 * microseconds (0 when taken from the cache), whether it came from the
 * cache (1) or from tuning (0), and the capture form: the layers of each
 * stage are independent, so they can run as concurrent branches of the
 * graph (forked onto side streams of default priority and joined back);
 * the plan replays both forms and keeps the faster, unless a cache line
 * "key blocks chunk us branches" pins it. Layers of at most 8 input channels, and
 * layers with several 64-row output tiles and at most 256 input channels, run
 * on their own kernels after the shared persistent launch of the others; the
 * schedule concerns the shared launch (a plan of such layers only has nothing
 * to tune and reports from_cache = 0). */
typedef struct ensei_schedule {
    int blocks;
    int from_cache;
    int64_t chunk;
    double homconv_us;
    int shared_layers;   /* layers in the shared persistent launch */
    int own_layers;      /* layers on a HomConv kernel of their own (narrow inputs, deep layers) */
    int branches;        /* 1: each stage's layers run as concurrent graph branches, 0: in order */
    int pad;
    double serial_us;    /* measured replay of the plan with the layers in order (0 if not timed) */
    double branches_us;  /* the same with concurrent branches (0 if not timed) */
} ensei_schedule;

/* Creates a plan for nlayers (1..ENSEI_MAX_PLAN_LAYERS) layers. Allocates the
 * transformed and packed filters and a small launch table on the context's
 * device (freed by ensei_plan_destroy), runs the filters' preparation, tunes
 * the schedule, runs the whole stack once eagerly (so every argument check of
 * the single calls applies and is reported here) and captures the graph.
 * Synchronous; it first waits for every piece of work already queued on the
 * device, so the layers' inputs may come from pending work on any stream. Errors: those of the single calls, ENSEI_ERR_LIMIT for too
 * many layers, ENSEI_ERR_HIP for allocation or capture failures. */
#define ENSEI_MAX_PLAN_LAYERS 64
int ensei_plan_create(ensei_ctx *ctx, const ensei_layer *layers, int nlayers, const char *tune_cache,
                      ensei_plan **out);

/* The same plan on seeded ciphertexts (ensei_encrypt_seeded,
 * ensei_homconv_seeded): each layer's ct_in holds only the b words, uint64
 * [batch][F][Cin], and HomConv regenerates the a-words from the layer's
 * seed_a. Every other buffer, and every result (ct_out, m, s_a, s_b), is
 * as in ensei_plan_create. Tuning-cache keys carry "/seeded". */
int ensei_plan_create_seeded(ensei_ctx *ctx, const ensei_layer *layers, int nlayers, const char *tune_cache,
                             ensei_plan **out);

/* Enqueues one run of the captured graph on `stream` (asynchronous). */
int ensei_plan_run(ensei_plan *plan, void *stream);

/* Enqueues one stage of a run, each captured as a graph of its own: 0 the
 * client's NTT2D and Enc of every layer, 1 the server's HomConv of every
 * layer (the shared persistent launch and the layers' own kernels), 2 Dec,
 * INTT2D and the server's share of every layer. Stages 0, 1, 2 in that order
 * on one stream are one ensei_plan_run (the two parties' steps can so be
 * enqueued, and timed, separately). ENSEI_ERR_ARG for another stage. */
int ensei_plan_run_stage(ensei_plan *plan, int stage, void *stream);

/* The schedule the plan runs (see ensei_schedule). */
int ensei_plan_schedule(const ensei_plan *plan, ensei_schedule *out);

/* Frees the plan's device memory and graph; NULL is accepted. Wait for the
 * plan's runs to finish first. */
int ensei_plan_destroy(ensei_plan *plan);

/* ------------------------------------------------------------ serving --
 * A server runs secure-convolution requests (the start round of Fig. 2 for
 * one image) of mixed shapes with continuous batching. A worker thread
 * admits queued requests in arrival order while their ciphertext state fits
 * the free part of a device budget, groups them into a batch and enqueues it
 * on one of `nstreams` streams (default priority): per request NTT2D and Enc,
 * one persistent HomConv launch over the tiles of every request of the batch
 * (requests of narrow-input or deep shapes run their own HomConv kernels),
 * then per request Dec, INTT2D and the server's share. Batches on different
 * streams overlap on the device; when a batch completes, its memory returns
 * to the budget and waiting requests are admitted. A request's ciphertexts
 * (x^, ct_in, ct_out, m: ensei_request_bytes) live in the server's budget
 * from admission to completion and never leave the device. Results are
 * bit-identical to the single calls on the same inputs, alone or in a mix.
 *
 * The server's filters of each shape are prepared once by
 * ensei_server_add_shape. A request's inputs and outputs are the caller's
 * device buffers: x [Cin][H][W] residues < p, s [n] ternary, e [Cin][F]
 * int32, r [Cout][F] masks < p, and the written shares s_a, s_b
 * [Cout][H][W]; the inputs must be complete in the order of the request's
 * `stream` and every buffer must stay valid
 * until the request has finished (done, failed or cancelled). Word j of
 * ciphertext (c, f) is keyed by seed_a and q = f*Cin + c, as ensei_encrypt
 * with one image and ct_index0 = 0.
 *
 * The server allocates its budget, launch tables and per-shape filters on the
 * context's device (at create / add_shape; nothing while serving). All calls
 * are thread-safe. Times are seconds since the server was created. */
typedef struct ensei_server ensei_server;

typedef struct ensei_shape {
    int H, W, Cin, Cout, kh, kw, n;
} ensei_shape;

typedef struct ensei_request {
    const uint32_t *x;
    const int8_t *s;
    const int32_t *e;
    const uint32_t *r;
    uint64_t seed_a;
    uint32_t *s_a;
    uint32_t *s_b;
    /* The hipStream_t (as void*; NULL = the null stream) whose queued work
     * produces x, s, e and r: the request's kernels start only after the
     * work queued on it before the submit (an event recorded there). */
    void *stream;
} ensei_request;

/* state: 0 queued, 1 running, 2 done, 3 failed (status holds the error),
 * 4 cancelled (status ENSEI_ERR_CANCELLED). */
typedef struct ensei_request_info {
    int state;
    int status;
    double t_submit, t_start, t_done;
} ensei_request_info;

typedef struct ensei_server_info {
    uint64_t budget_bytes, used_bytes, peak_used_bytes;
    uint64_t queued, inflight_batches, completed, failed, batches;
    uint64_t cancelled, refused; /* cancel calls that took effect; submits refused with ENSEI_ERR_BUDGET */
} ensei_server_info;

/* Device bytes of one request of this shape inside the budget (0 if invalid). */
size_t ensei_request_bytes(const ensei_shape *shape);

/* budget_bytes of ciphertext state; 1 <= nstreams <= 8; 1 <= max_batch <= 256
 * requests per batch. Starts the worker thread. */
int ensei_server_create(ensei_ctx *ctx, size_t budget_bytes, int nstreams, int max_batch, ensei_server **out);

/* The same server on seeded ciphertexts (ensei_encrypt_seeded,
 * ensei_homconv_seeded): a request keeps only the b words of its input
 * ciphertexts, so it takes 8*F*n*Cin bytes less of the budget than
 * ensei_request_bytes states (up to alignment); results are unchanged. */
int ensei_server_create_seeded(ensei_ctx *ctx, size_t budget_bytes, int nstreams, int max_batch,
                               ensei_server **out);

/* Registers a shape with the server's filters w [Cout][Cin][kh][kw] int32
 * (read once, synchronously, after every piece of work already queued on the
 * device has finished, so w may come from pending work on any stream).
 * ENSEI_ERR_BUDGET if one request of the shape does not fit the budget; the
 * single calls' shape errors otherwise. */
int ensei_server_add_shape(ensei_server *server, const ensei_shape *shape, const int32_t *w, int *shape_id);

/* Queues one request; returns at once with its ticket. Its arrival time is
 * taken before the call waits for the server's lock. ENSEI_ERR_BUDGET (and
 * nothing queued) if its footprint exceeds the budget, or if the footprints
 * of the requests waiting for admission would exceed the queue limit. */
int ensei_server_submit(ensei_server *server, int shape_id, const ensei_request *req, uint64_t *ticket);

/* Cancels a request (paper Fig. 2: the client may abandon a round). A queued
 * request leaves the queue at once: it never takes budget or device time,
 * and requests behind it may be admitted in its place. A running request's
 * device work cannot be recalled: it is marked, its budget returns when its
 * batch has finished, and it is then reported cancelled (its output shares
 * may or may not have been written). Other requests are not affected. Returns
 * ENSEI_OK, ENSEI_ERR_ARG for an unknown ticket, ENSEI_ERR_STATE if the
 * request has already finished. */
int ensei_server_cancel(ensei_server *server, uint64_t ticket);

/* Caps the bytes of requests waiting for admission (0 = no cap, the
 * default); a submit past the cap returns ENSEI_ERR_BUDGET. */
int ensei_server_set_queue_limit(ensei_server *server, size_t bytes);

/* The server's clock: seconds since it was created (the time base of
 * ensei_request_info). */
int ensei_server_clock(ensei_server *server, double *now);

/* The request's state and times (ENSEI_ERR_ARG for an unknown ticket). */
int ensei_server_poll(ensei_server *server, uint64_t ticket, ensei_request_info *info);

/* Blocks until the request has finished (timeout_ms < 0: no limit); returns
 * its status (ENSEI_ERR_CANCELLED for a cancelled one), or ENSEI_ERR_TIMEOUT. */
int ensei_server_wait(ensei_server *server, uint64_t ticket, int timeout_ms);

/* Drops a finished request's record (ENSEI_ERR_ARG if unknown or not done). */
int ensei_server_forget(ensei_server *server, uint64_t ticket);

/* Budget use (now and peak), queue length, batches in flight and counts. */
int ensei_server_stats(ensei_server *server, ensei_server_info *out);

/* Finishes every queued and running request, then frees the server. */
int ensei_server_destroy(ensei_server *server);

#ifdef __cplusplus
}
#endif

#endif /* ENSEI_H */
