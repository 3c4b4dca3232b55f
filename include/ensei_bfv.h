/*
 * ensei_bfv.h — the packed (BFV / RLWE) instantiation of ENSEI's secure
 * convolution on one MI355X, part of libensei.so.
 *
 * The paper instantiates its protocol with packed BFV (Sec. 3.1, Eq.
 * (bfv_enc); Sec. 5.1, Fig. "Modified Enc-SIMDScMult-Dec"; Sec. 5.2 and
 * Table 2's parameter sets, n = 2048). Here, with R = Z[X]/(X^n + 1):
 *   - t (Table 2's p_E) is a prime = 1 mod 2n: a plaintext holds n slots, a
 *     slot vector v stands for the polynomial u = INTT_t(v), and slot-wise
 *     products are products in R mod t;
 *   - q = q0 q1, two primes = 1 mod 2n below 2^30 (residue number system),
 *     Delta = q / t rounded to the nearest integer (q / p_E of Eq. (bfv_enc)),
 *     so that Delta t = q - rho with |rho| <= t/2; limbs with a small |rho|
 *     keep the noise of a plaintext product small;
 *   - the negacyclic transform mod a prime m evaluates a polynomial at the
 *     odd powers of psi_m = g^((m-1)/2n), g the smallest primitive root of m:
 *     NTT_m(u)[k] = sum_j u_j psi^((2k+1) j) (natural order k);
 *   - a ciphertext is held in evaluation form, per limb l the pair
 *     (a^, b^) with b^ = a^ . s^ + NTT_q(Delta u + e) (the paper's
 *     (c0, c1) = (-a, a s + (q/p_E) u + e) with c0 = -a), s^ = NTT_q(s) for a
 *     ternary key s; the public a^ of limb l, slot k of ciphertext c is
 *     SplitMix64 output ((c0 + c) 2 + l) n + k + 1 of seed_a, mod q_l (the
 *     constants generated offline of Sec. 5.1);
 *   - a ciphertext array is uint32 [count][2 limbs][2 words: a^, b^][n].
 *
 * Packing of one layer (B images, C channels, F = H W spectra of ensei_ntt2d
 * mod t): with F <= n a slot vector holds P = n / F channels, channel g P + j
 * at slots [j F, (j+1) F) of vector g; with F > n a channel spans K = F / n
 * vectors, chunk k holding frequencies [k n, (k+1) n). G = ceil(C / P)
 * vectors per chunk; vector (b, g, k) has index (b G + g) K + k. Unused slots
 * are 0. HomConv's output vector (o, k) holds in slot block j the sum over
 * the input channels g P + j; the client adds the blocks (ensei_bfv_fold),
 * so no rotation is needed anywhere (the point of Sec. 4).
 *
 * Common rules are those of ensei.h: device pointers owned by the caller,
 * asynchronous calls on `stream`, host-side checks before any launch and a
 * negative ENSEI_ERR_* on error; the current device must be the context's.
 */
#ifndef ENSEI_BFV_H
#define ENSEI_BFV_H

#include <stddef.h>
#include <stdint.h>

#include "ensei.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ensei_bfv_ctx ensei_bfv_ctx;

/* Creates a context for (t, q0, q1, n) on `device`: n a power of two in
 * [16, 4096]; t, q0, q1 distinct primes = 1 mod 2n, each below 2^30
 * (ENSEI_ERR_MODULUS otherwise; ENSEI_ERR_ARG for n). Uploads the twiddle
 * tables of the three moduli (a few tens of KB); the only allocating call. */
int ensei_bfv_ctx_create(ensei_bfv_ctx **out, uint32_t t, uint32_t q0, uint32_t q1, int n, int device);
int ensei_bfv_ctx_destroy(ensei_bfv_ctx *ctx);

/* The key in evaluation form: s_hat uint32 [2 limbs][2][n], entry [l][0][k]
 * = NTT_{q_l}(s)[k] and [l][1][k] its multiplier companion
 * floor(s^ 2^32 / q_l); s: int8 [n] in {-1, 0, 1}. */
int ensei_bfv_key(ensei_bfv_ctx *ctx, const int8_t *s, uint32_t *s_hat, void *stream);

/* Client: packs the spectra x_hat uint32 [B][C][F] (values < t) into slot
 * vectors as above and encrypts every vector (Eq. (bfv_enc) in evaluation
 * form, the image's spectrum embedded straight into the slots as in Sec.
 * 5.1): ct uint32 [B G K][2][2][n]; e int32 [B G K][n] the coefficient-domain
 * errors; s_hat from ensei_bfv_key; vector c takes the public a^ of
 * ciphertext index ct_index0 + c. F a power of two dividing n, or a multiple
 * of n. */
int ensei_bfv_encrypt(ensei_bfv_ctx *ctx, const uint32_t *x_hat, int64_t B, int C, int64_t F, const uint32_t *s_hat,
                      const int32_t *e, uint64_t seed_a, uint64_t ct_index0, uint32_t *ct, void *stream);

/* Server setup: the filters W^ uint32 [Cout][Cin][F] (values < t, the
 * transforms of ensei_weight_prep mod t) as plaintext multipliers, packed
 * like the inputs (slot block j of vector (o, g, k) holds W^[o][g P + j]),
 * encoded unscaled (coefficients INTT_t lifted to (-t/2, t/2]) and
 * transformed: w_enc uint32 [Cout][G][K][2 limbs][2][n] (value, companion
 * floor(w 2^32 / q_l)). */
int ensei_bfv_encode_filters(ensei_bfv_ctx *ctx, const uint32_t *w_hat, int Cout, int Cin, int64_t F,
                             uint32_t *w_enc, void *stream);

/* Server: HomShare's masks as trivial encryptions: r uint32 [count][n] slot
 * vectors (values < t) -> mask_enc uint32 [count][2 limbs][n] =
 * NTT_{q_l}(Delta INTT_t(r)), the b^ word of an encryption of r with a^ = 0
 * and no error. */
int ensei_bfv_encode_masks(ensei_bfv_ctx *ctx, const uint32_t *r, int64_t count, uint32_t *mask_enc, void *stream);

/* Server: SIMDScMult with the filters, the sum over input vectors and the
 * masks (Fig. 2's Hadamard product, channel sum and HomShare on packed
 * ciphertexts): for image b, output o, chunk k, limb l and word w,
 *   ct_out[(b Cout + o) K + k][l][w][s] = sum_g w_enc[o][g][k][l][0][s]
 *        * ct_in[(b G + g) K + k][l][w][s]  mod q_l,
 * and the b^ word gains mask_enc[(b Cout + o) K + k][l][s]. ct_out uint32
 * [B Cout K][2][2][n]. Cin, F give G and K as above. */
int ensei_bfv_homconv(ensei_bfv_ctx *ctx, const uint32_t *ct_in, const uint32_t *w_enc, const uint32_t *mask_enc,
                      int64_t B, int Cin, int Cout, int64_t F, uint32_t *ct_out, void *stream);

/* Client: decryption of `count` ciphertexts ct [count][2][2][n] to slot
 * vectors v uint32 [count][n]: phi = INTT_q(b^ - a^ . s^) per limb, joined
 * by the Chinese remainder theorem, m_j = floor((t phi_j + (q-1)/2) / q) mod
 * t, v = NTT_t(m). */
int ensei_bfv_decrypt(ensei_bfv_ctx *ctx, const uint32_t *ct, const uint32_t *s_hat, int64_t count, uint32_t *v,
                      void *stream);

/* Circuit privacy (Sec. 4.1 leaves it to Gazelle's treatment): re-randomises
 * `count` ciphertexts ct [count][2][2][n] in place by adding to each a fresh
 * public-key encryption of zero, (a^_pk rho^ + e1^, b^_pk rho^ + e2^) per
 * limb, so that the a^ word is a fresh RLWE sample rather than a sum the
 * client could divide by its inputs, and e2 floods the noise that depends on
 * the filters. pk uint32 [2][2][n] is the client's public key: its
 * encryption of an all-zero spectrum (ensei_bfv_encrypt). The server's draws
 * for ciphertext ct_index0 + i and coefficient j: z = SplitMix64 output
 * ((ct_index0 + i) 3 + w) n + j + 1 of seed_r, value
 * floor(hi32(z) (2B + 1) / 2^32) - B, with w = 0: rho (B = 1), w = 1: e1
 * (B = 16), w = 2: e2 (B = flood). The decryption is unchanged while the
 * total noise stays below Delta / 2; flood < 2^31 (ENSEI_ERR_ARG). */
int ensei_bfv_rerandomize(ensei_bfv_ctx *ctx, uint32_t *ct, int64_t count, const uint32_t *pk, uint64_t seed_r,
                          uint64_t ct_index0, uint32_t flood, void *stream);

/* The fold of slot vectors v [B][C K][n] back to spectra y uint32 [B][C][F]:
 * y[b][c][f] = sum of the P slot blocks (F <= n) or chunk f / n (F > n),
 * mod t; negate = 1 gives -y mod t (the server's share of the masks). The
 * client folds its decrypted outputs; the server folds its masks. */
int ensei_bfv_fold(ensei_bfv_ctx *ctx, const uint32_t *v, int64_t B, int C, int64_t F, int negate, uint32_t *y,
                   void *stream);

/* Sizes: G and K of the packing (slot vectors per chunk and chunks per
 * channel) for C channels of F spectra; returns G * K, or 0 for invalid
 * sizes. */
int64_t ensei_bfv_vectors(const ensei_bfv_ctx *ctx, int C, int64_t F);

#ifdef __cplusplus
}
#endif

#endif /* ENSEI_BFV_H */
