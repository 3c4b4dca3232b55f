/*
 * CPU oracle for the packed (BFV / RLWE) instantiation of ENSEI's secure
 * convolution (Bian et al., CVPR 2020, Sec. 3.1 and Sec. 5).
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, obviously correct
 * restatement of what the packed path computes: every transform is its
 * defining sum, O(n^2). Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it. It shares no code, header, table
 * or constant generator with the GPU library and never links it.
 *
 * Conventions (readings of the paper, each listed with its reason in the
 * design notes):
 *   - ring R = Z[X]/(X^n + 1), n a power of two (n = 2048 in Table 2);
 *   - plaintext modulus t (Table 2's p_E), a prime with t = 1 mod 2n, so that
 *     X^n + 1 splits mod t and a plaintext holds n slots (Sec. 3.1 packing);
 *     the image transform and the shares use the same t;
 *   - ciphertext modulus q = q_0 q_1, two primes q_l = 1 mod 2n (residue
 *     number system), Delta = q / t rounded to the nearest integer (Eq.
 *     (bfv_enc) writes q / p_E, which is not an integer; with the limbs
 *     chosen for a small centred q mod t, Delta t = q - rho with |rho| small,
 *     and rho is what multiplies the wrap term of a plaintext product);
 *   - psi_m = g^((m - 1) / 2n) for g the smallest primitive root of the prime
 *     m: a primitive 2n-th root of unity, psi^n = -1;
 *   - the negacyclic transform of a length-n vector mod m evaluates its
 *     polynomial at the odd powers of psi (a ring isomorphism
 *     Z_m[X]/(X^n+1) -> Z_m^n):  NTT(u)[k] = sum_j u_j psi^((2k+1) j),
 *     inverse INTT(v)[j] = n^-1 sum_k v_k psi^(-(2k+1) j); slot-wise
 *     products are negacyclic convolutions of coefficients;
 *   - slot encoding: a slot vector v in Z_t^n is the plaintext polynomial
 *     u = INTT_t(v) (coefficients in [0, t)); decoding is NTT_t;
 *   - ciphertexts are held in evaluation form per limb: (a^, b^) with
 *     b^ = a^ . s^ + NTT_q(Delta u + e) (the paper's (c0, c1) = (-a, a s +
 *     (q/p_E) u + e) with c0 = -a), s^ = NTT_q(s) for a ternary key s; the
 *     public a^ comes straight from a counter-based generator in evaluation
 *     form (the constants generated offline of Sec. 5.1): limb l, slot k of
 *     ciphertext index c is SplitMix64 output ((c0 + c) L + l) n + k + 1 of
 *     seed_a, reduced mod q_l;
 *   - a plaintext that multiplies a ciphertext (SIMDScMult, Sec. 3.1) is
 *     encoded unscaled: its coefficients INTT_t(w) lifted to the centred
 *     range (-t/2, t/2], then transformed mod q_l;
 *   - decryption: phi = INTT_q(b^ - a^ . s^) per limb, joined by the Chinese
 *     remainder theorem to [0, q), m_j = floor((t phi_j + (q - 1) / 2) / q)
 *     mod t (round to nearest), slots = NTT_t(m).
 *
 * Arrays of residues mod q_l are uint32 (q_l < 2^31); a ciphertext is
 * [L][2][n] (limb, word 0 = a^, word 1 = b^, slot).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define NLIMB 2

static uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

static uint64_t powm(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulm(r, a, m);
        a = mulm(a, a, m);
        e >>= 1;
    }
    return r;
}

int bo_is_prime(uint64_t m) {
    if (m < 2) return 0;
    for (uint64_t d = 2; d * d <= m; ++d)
        if (m % d == 0) return 0;
    return 1;
}

/* Smallest generator of the multiplicative group of Z_m (m prime). */
static uint64_t primitive_root(uint64_t m) {
    uint64_t r = m - 1, fac[64];
    int nf = 0;
    for (uint64_t d = 2; d * d <= r; ++d) {
        if (r % d == 0) {
            fac[nf++] = d;
            while (r % d == 0) r /= d;
        }
    }
    if (r > 1) fac[nf++] = r;
    for (uint64_t g = 2; g < m; ++g) {
        int ok = 1;
        for (int i = 0; i < nf && ok; ++i)
            if (powm(g, (m - 1) / fac[i], m) == 1) ok = 0;
        if (ok) return g;
    }
    return 0;
}

/* psi: a primitive 2n-th root of unity mod the prime m (0 if 2n does not
 * divide m - 1). */
uint64_t bo_psi(uint64_t m, int n) {
    uint64_t two_n = 2 * (uint64_t)n;
    if (n < 1 || (m - 1) % two_n != 0) return 0;
    return powm(primitive_root(m), (m - 1) / two_n, m);
}

uint64_t bo_splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Negacyclic transform of `batch` vectors of length n mod m, by its
 * defining sum. forward: out[k] = sum_j in[j] psi^((2k+1) j);
 * inverse: out[j] = n^-1 sum_k in[k] psi^(-(2k+1) j). */
void bo_negacyclic(uint64_t m, int n, int64_t batch, const uint32_t *in, uint32_t *out, int inverse) {
    uint64_t psi = bo_psi(m, n);
    if (inverse) psi = powm(psi, m - 2, m);
    const uint64_t two_n = 2 * (uint64_t)n;
    uint64_t *pw = malloc(two_n * sizeof *pw); /* psi^e for e < 2n (psi has order 2n) */
    pw[0] = 1;
    for (uint64_t e = 1; e < two_n; ++e) pw[e] = mulm(pw[e - 1], psi, m);
    const uint64_t scale = inverse ? powm((uint64_t)n, m - 2, m) : 1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < batch; ++t) {
        const uint32_t *x = in + t * n;
        for (int k = 0; k < n; ++k) { /* output index k, input index j */
            uint64_t acc = 0;
            for (int j = 0; j < n; ++j) {
                const uint64_t e = inverse ? (uint64_t)(2 * j + 1) * k : (uint64_t)(2 * k + 1) * j;
                acc = (acc + mulm(x[j] % m, pw[e % two_n], m)) % m;
            }
            out[t * n + k] = (uint32_t)mulm(acc, scale, m);
        }
    }
    free(pw);
}

/* q = q0 q1 and Delta = the integer nearest to q / t (t is odd: no ties). */
static u128 modulus_q(const uint64_t *qs) { return (u128)qs[0] * qs[1]; }
static u128 delta_q(uint64_t t, const uint64_t *qs) { return (modulus_q(qs) + t / 2) / t; }

/* Delta mod q_l for l < 2 (host helper for callers). */
uint64_t bo_delta_mod(uint64_t t, uint64_t q0, uint64_t q1, int l) {
    const uint64_t qs[NLIMB] = {q0, q1};
    return (uint64_t)(delta_q(t, qs) % qs[l]);
}

/* The plaintext-side encodings of slot vectors v[batch][n] (values < t),
 * into evaluation form [batch][L][n] mod q_l:
 *   scaled = 1: NTT_q(Delta * INTT_t(v)) with the coefficients in [0, t)
 *               (a trivial encryption's b^: HomShare's mask Delta r);
 *   scaled = 0: NTT_q(lift(INTT_t(v))) with the coefficients lifted to
 *               (-t/2, t/2] (a plaintext multiplier: the filters). */
void bo_encode(uint64_t t, uint64_t q0, uint64_t q1, int n, int64_t batch, const uint32_t *v, int scaled,
               uint32_t *out) {
    const uint64_t qs[NLIMB] = {q0, q1};
    uint32_t *u = malloc((size_t)batch * n * sizeof *u);
    uint32_t *c = malloc((size_t)batch * n * sizeof *c);
    bo_negacyclic(t, n, batch, v, u, 1);
    for (int l = 0; l < NLIMB; ++l) {
        const uint64_t m = qs[l], dl = (uint64_t)(delta_q(t, qs) % m);
        for (int64_t i = 0; i < batch * n; ++i) {
            uint64_t x = u[i];
            if (scaled)
                x = mulm(dl, x, m);
            else if (x > t / 2)
                x = m - (t - x); /* centred lift of x - t */
            c[i] = (uint32_t)(x % m);
        }
        uint32_t *tmp = malloc((size_t)batch * n * sizeof *tmp);
        bo_negacyclic(m, n, batch, c, tmp, 0);
        for (int64_t b = 0; b < batch; ++b) memcpy(out + (b * NLIMB + l) * n, tmp + b * n, n * sizeof *out);
        free(tmp);
    }
    free(u);
    free(c);
}

/* The key in evaluation form: s_hat[L][n] = NTT_q(s mod q_l). */
void bo_key(uint64_t q0, uint64_t q1, int n, const int8_t *s, uint32_t *s_hat) {
    const uint64_t qs[NLIMB] = {q0, q1};
    uint32_t *c = malloc(n * sizeof *c);
    for (int l = 0; l < NLIMB; ++l) {
        for (int j = 0; j < n; ++j) c[j] = (uint32_t)(s[j] < 0 ? qs[l] - 1 : (uint64_t)s[j]);
        bo_negacyclic(qs[l], n, 1, c, s_hat + l * n, 0);
    }
    free(c);
}

/* Enc of `count` slot vectors v[count][n] (values < t) under the ternary key
 * s with errors e[count][n] (coefficient domain): ct[count][L][2][n]. */
void bo_encrypt(uint64_t t, uint64_t q0, uint64_t q1, int n, int64_t count, const uint32_t *v, const int8_t *s,
                const int32_t *e, uint64_t seed_a, uint64_t ct_index0, uint32_t *ct) {
    const uint64_t qs[NLIMB] = {q0, q1};
    uint32_t *u = malloc((size_t)count * n * sizeof *u);
    uint32_t *c = malloc((size_t)count * n * sizeof *c);
    uint32_t *ch = malloc((size_t)count * n * sizeof *ch);
    uint32_t *s_hat = malloc((size_t)NLIMB * n * sizeof *s_hat);
    bo_key(q0, q1, n, s, s_hat);
    bo_negacyclic(t, n, count, v, u, 1);
    for (int l = 0; l < NLIMB; ++l) {
        const uint64_t m = qs[l], dl = (uint64_t)(delta_q(t, qs) % m);
        for (int64_t i = 0; i < count * n; ++i) {
            const uint64_t ei = e[i] < 0 ? m - (uint64_t)(-(int64_t)e[i]) % m : (uint64_t)e[i] % m;
            c[i] = (uint32_t)((mulm(dl, u[i], m) + ei) % m);
        }
        bo_negacyclic(m, n, count, c, ch, 0);
        for (int64_t i = 0; i < count; ++i)
            for (int k = 0; k < n; ++k) {
                const uint64_t a = bo_splitmix64(seed_a, ((ct_index0 + (uint64_t)i) * NLIMB + (uint64_t)l) * (uint64_t)n +
                                                             (uint64_t)k + 1) % m;
                uint32_t *w = ct + ((i * NLIMB + l) * 2) * (int64_t)n;
                w[k] = (uint32_t)a;
                w[n + k] = (uint32_t)((mulm(a, s_hat[l * n + k], m) + ch[i * n + k]) % m);
            }
    }
    free(u);
    free(c);
    free(ch);
    free(s_hat);
}

/* Decryption phase in coefficients: phi[count][n] in [0, q) (uint64, q <
 * 2^64) of ct[count][L][2][n]: INTT_q(b^ - a^ . s^) per limb, joined by the
 * Chinese remainder theorem. */
void bo_phase(uint64_t q0, uint64_t q1, int n, int64_t count, const uint32_t *ct, const int8_t *s, uint64_t *phi) {
    const uint64_t qs[NLIMB] = {q0, q1};
    uint32_t *s_hat = malloc((size_t)NLIMB * n * sizeof *s_hat);
    uint32_t *d = malloc((size_t)count * n * sizeof *d);
    uint32_t *r[NLIMB];
    bo_key(q0, q1, n, s, s_hat);
    for (int l = 0; l < NLIMB; ++l) {
        const uint64_t m = qs[l];
        for (int64_t i = 0; i < count; ++i)
            for (int k = 0; k < n; ++k) {
                const uint32_t *w = ct + ((i * NLIMB + l) * 2) * (int64_t)n;
                d[i * n + k] = (uint32_t)((w[n + k] + m - mulm(w[k], s_hat[l * n + k], m)) % m);
            }
        r[l] = malloc((size_t)count * n * sizeof *r[l]);
        bo_negacyclic(m, n, count, d, r[l], 1);
    }
    /* x = r0 + q0 ((r1 - r0) q0^-1 mod q1) */
    const uint64_t inv = powm(q0 % q1, q1 - 2, q1);
    for (int64_t i = 0; i < count * n; ++i) {
        const uint64_t h = mulm((r[1][i] + q1 - r[0][i] % q1) % q1, inv, q1);
        phi[i] = (uint64_t)((u128)r[0][i] + (u128)q0 * h);
    }
    for (int l = 0; l < NLIMB; ++l) free(r[l]);
    free(s_hat);
    free(d);
}

/* Dec: slots v[count][n] of ct[count][L][2][n]. */
void bo_decrypt(uint64_t t, uint64_t q0, uint64_t q1, int n, int64_t count, const uint32_t *ct, const int8_t *s,
                uint32_t *v) {
    const uint64_t qs[NLIMB] = {q0, q1};
    const u128 q = modulus_q(qs);
    uint64_t *phi = malloc((size_t)count * n * sizeof *phi);
    uint32_t *mc = malloc((size_t)count * n * sizeof *mc);
    bo_phase(q0, q1, n, count, ct, s, phi);
    for (int64_t i = 0; i < count * n; ++i) mc[i] = (uint32_t)((((u128)phi[i] * t + (q - 1) / 2) / q) % t);
    bo_negacyclic(t, n, count, mc, v, 0);
    free(phi);
    free(mc);
}

/* Packing of B images' spectra x_hat[B][C][F] (values < t) into slot
 * vectors. With F <= n each vector holds P = n / F channels (channel g P + j
 * at slots [j F, (j+1) F)), with F > n a channel spans K = F / n vectors
 * (chunk k at slots [0, n) holds frequencies [k n, (k+1) n)); vector index
 * (b, g, k) -> (b G + g) K + k for G = ceil(C / P). Unused slots are 0. */
void bo_pack(int64_t B, int C, int64_t F, int n, const uint32_t *x_hat, uint32_t *v) {
    const int64_t P = F <= n ? n / F : 1, K = F <= n ? 1 : F / n, G = (C + P - 1) / P, Fp = F <= n ? F : n;
    memset(v, 0, (size_t)(B * G * K) * n * sizeof *v);
    for (int64_t b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int64_t f = 0; f < F; ++f) {
                const int64_t g = c / P, j = c % P, k = f / Fp, slot = j * Fp + f % Fp;
                v[((b * G + g) * K + k) * n + slot] = x_hat[(b * C + c) * F + f];
            }
}

/* The server's filter plaintexts: for output o, input vector g and chunk k,
 * the slot vector holding W^[o][g P + j][f] where the packing puts x^[g P +
 * j][f]; encoded unscaled (bo_encode): w_enc[Cout][G][K][L][n]. */
void bo_filters(uint64_t t, uint64_t q0, uint64_t q1, int Cout, int Cin, int64_t F, int n, const uint32_t *w_hat,
                uint32_t *w_enc) {
    const int64_t P = F <= n ? n / F : 1, K = F <= n ? 1 : F / n, G = (Cin + P - 1) / P, Fp = F <= n ? F : n;
    uint32_t *v = calloc((size_t)(Cout * G * K) * n, sizeof *v);
    for (int o = 0; o < Cout; ++o)
        for (int c = 0; c < Cin; ++c)
            for (int64_t f = 0; f < F; ++f) {
                const int64_t g = c / P, j = c % P, k = f / Fp, slot = j * Fp + f % Fp;
                v[(((int64_t)o * G + g) * K + k) * n + slot] = w_hat[((int64_t)o * Cin + c) * F + f];
            }
    bo_encode(t, q0, q1, n, Cout * G * K, v, 0, w_enc);
    free(v);
}

/* SIMDScMult, the channel sum and HomShare (Fig. 2 with packed
 * ciphertexts): for image b, output o, chunk k, limb l, word w, slot s,
 *   ct_out[b][o][k][l][w][s] = sum_g w_enc[o][g][k][l][s] ct_in[b][g][k][l][w][s] mod q_l,
 * then the b^ word gains mask_enc[b][o][k][l][s] (the scaled encoding of the
 * server's masks, bo_encode with scaled = 1). ct_in [B][G K][L][2][n],
 * ct_out [B][Cout K][L][2][n]. */
void bo_homconv(uint64_t q0, uint64_t q1, int64_t B, int G, int Cout, int K, int n, const uint32_t *ct_in,
                const uint32_t *w_enc, const uint32_t *mask_enc, uint32_t *ct_out) {
    const uint64_t qs[NLIMB] = {q0, q1};
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; ++b)
        for (int o = 0; o < Cout; ++o)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < NLIMB; ++l)
                    for (int w = 0; w < 2; ++w)
                        for (int s = 0; s < n; ++s) {
                            const uint64_t m = qs[l];
                            uint64_t acc = 0;
                            for (int g = 0; g < G; ++g) {
                                const uint64_t wv = w_enc[((((int64_t)o * G + g) * K + k) * NLIMB + l) * n + s];
                                const uint64_t cv = ct_in[((((b * G + g) * K + k) * NLIMB + l) * 2 + w) * n + s];
                                acc = (acc + mulm(wv, cv, m)) % m;
                            }
                            if (w == 1) acc = (acc + mask_enc[(((b * Cout + o) * K + k) * NLIMB + l) * n + s]) % m;
                            ct_out[((((b * Cout + o) * K + k) * NLIMB + l) * 2 + w) * n + s] = (uint32_t)acc;
                        }
}

/* The client's fold of decrypted output slots v[B][Cout K][n] back to
 * spectra y[B][Cout][F]: y[b][o][f] = sum over the P slot blocks of the
 * packing, mod t (each block holds the partial sum over one residue class of
 * input channels, and the mask's blocks add up to the server's total mask). */
void bo_fold(uint64_t t, int64_t B, int Cout, int64_t F, int n, const uint32_t *v, uint32_t *y) {
    const int64_t P = F <= n ? n / F : 1, K = F <= n ? 1 : F / n, Fp = F <= n ? F : n;
    for (int64_t b = 0; b < B; ++b)
        for (int o = 0; o < Cout; ++o)
            for (int64_t f = 0; f < F; ++f) {
                const int64_t k = f / Fp;
                uint64_t acc = 0;
                for (int64_t j = 0; j < P; ++j) acc += v[((b * Cout + o) * K + k) * n + j * Fp + f % Fp];
                y[(b * Cout + o) * F + f] = (uint32_t)(acc % t);
            }
}

/* ------------------------------------------------- circuit privacy --- */

/* The server's randomness for re-randomising output ciphertext c0 + i
 * (i < count): for w = 0 (rho), 1 (e1), 2 (e2) and coefficient j,
 * z = SplitMix64 output ((c0 + i) 3 + w) n + j + 1 of seed_r, and the draw is
 * floor(hi32(z) (2 B + 1) / 2^32) - B with B = 1, E1_BOUND, flood for
 * w = 0, 1, 2 (a ternary rho, a small e1, the flooding e2). draws:
 * int32 [count][3][n]. */
#define E1_BOUND 16
void bo_rerand_draws(uint64_t seed_r, uint64_t ct_index0, int n, int64_t count, uint32_t flood, int32_t *draws) {
    for (int64_t i = 0; i < count; ++i)
        for (int w = 0; w < 3; ++w) {
            const uint64_t B = w == 0 ? 1 : w == 1 ? E1_BOUND : flood;
            for (int j = 0; j < n; ++j) {
                const uint64_t z = bo_splitmix64(seed_r, ((ct_index0 + (uint64_t)i) * 3 + (uint64_t)w) * (uint64_t)n +
                                                             (uint64_t)j + 1);
                draws[(i * 3 + w) * n + j] = (int32_t)((int64_t)(((z >> 32) * (2 * B + 1)) >> 32) - (int64_t)B);
            }
        }
}

/* Circuit privacy by re-randomisation (the paper defers it to Gazelle, Sec.
 * 4.1): every ciphertext of ct[count][L][2][n] gains a fresh public-key
 * encryption of zero, (a^_pk rho^ + e1^, b^_pk rho^ + e2^), with the
 * client's public key pk[L][2][n] (an encryption of zero under s:
 * b^_pk = a^_pk s^ + NTT(e_pk)) and the draws of bo_rerand_draws, each
 * transformed per limb. The message is unchanged; the a^ word becomes a fresh
 * RLWE sample, and e2 floods the noise. In place. */
void bo_rerandomize(uint64_t q0, uint64_t q1, int n, int64_t count, uint32_t *ct, const uint32_t *pk, uint64_t seed_r,
                    uint64_t ct_index0, uint32_t flood) {
    const uint64_t qs[NLIMB] = {q0, q1};
    int32_t *dr = malloc((size_t)count * 3 * n * sizeof *dr);
    uint32_t *c = malloc((size_t)count * 3 * n * sizeof *c);
    uint32_t *h = malloc((size_t)count * 3 * n * sizeof *h);
    bo_rerand_draws(seed_r, ct_index0, n, count, flood, dr);
    for (int l = 0; l < NLIMB; ++l) {
        const uint64_t m = qs[l];
        for (int64_t i = 0; i < count * 3 * n; ++i)
            c[i] = (uint32_t)(dr[i] < 0 ? m - (uint64_t)(-(int64_t)dr[i]) % m : (uint64_t)dr[i] % m) % m;
        bo_negacyclic(m, n, count * 3, c, h, 0);
        const uint32_t *pa = pk + (l * 2) * (int64_t)n, *pb = pa + n;
        for (int64_t i = 0; i < count; ++i) {
            uint32_t *wa = ct + ((i * NLIMB + l) * 2) * (int64_t)n, *wb = wa + n;
            const uint32_t *rho = h + (i * 3) * (int64_t)n, *e1 = rho + n, *e2 = e1 + n;
            for (int k = 0; k < n; ++k) {
                wa[k] = (uint32_t)((wa[k] + mulm(pa[k], rho[k], m) + e1[k]) % m);
                wb[k] = (uint32_t)((wb[k] + mulm(pb[k], rho[k], m) + e2[k]) % m);
            }
        }
    }
    free(dr);
    free(c);
    free(h);
}

int bo_set_threads(int k);
#ifdef _OPENMP
#include <omp.h>
int bo_set_threads(int k) {
    if (k > 0) omp_set_num_threads(k);
    return omp_get_max_threads();
}
#else
int bo_set_threads(int k) {
    (void)k;
    return 1;
}
#endif
