/*
 * CPU oracle for the frequency-domain secure convolution (FDSC) hot path of
 * ENSEI (Bian et al., CVPR 2020).
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, obviously correct
 * restatement of what the hot path computes. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it. It shares no code,
 * header, table or constant generator with the GPU library, and it never
 * imports or links it.
 *
 * Conventions (each one a reading of the paper, listed with its reason in the
 * design notes):
 *   - one prime p serves as NTT modulus, share modulus and plaintext modulus
 *     (Sec. 5.2 requires p_E >= p_A >= p_N; equality satisfies it);
 *   - the ciphertext modulus is q = 2^64, realised as uint64 wraparound;
 *   - the transform of an H x W channel is the cyclic 2D NTT of Eq.
 *     (ntt_transform_eq) applied along both axes, with omega_N = g^((p-1)/N)
 *     for g the smallest primitive root of p; flatten is row-major,
 *     f = k1 * W + k2 (Sec. 4.1, step "Line 1-3");
 *   - the inverse uses omega^-1 and multiplies by (H W)^-1 mod p;
 *   - encryption is LWE per frequency coefficient: ciphertext words
 *     [a_0 .. a_{n-1}, b] with b = <a, s> + Delta * m + e mod 2^64, which is
 *     the paper's (c0, c1) = (-a, a t + (q/p) u + e0) of Eq. (bfv_enc) with one
 *     coefficient per ciphertext; Delta = floor(2^64 / p);
 *   - storage (a layout the paper leaves open): the ciphertexts of channel c,
 *     frequency f, image b are stored word-major, word j at
 *     ct[b][f][j][c] (C channels innermost); ciphertext index
 *     q = (b F + f) C + c. With C = 1 this is a plain list of rows [N][n+1];
 *   - the a-words come from the SplitMix64 generator (Steele, Lea and Flood,
 *     OOPSLA 2014): word j of ciphertext q is output number
 *     (q0 + q) n + j + 1 of the generator seeded with seed_a;
 *   - HomConv: for every frequency f, ct_out[o,f] = sum_i W^[o,i,f] ct_in[i,f]
 *     mod 2^64 (the homomorphic Hadamard product with a plaintext, summed over
 *     input channels), then Delta * r[o,f] is added to the b word (HomShare,
 *     Eq. (homshare), with the server keeping -r as its share);
 *   - decryption rounds half up: m = floor((phi * p + 2^63) / 2^64) mod p for
 *     phi = b - <a, s> mod 2^64 (the round-off of Sec. 3.1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- Z_p --- */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod(r, a, p);
        a = mulmod(a, a, p);
        e >>= 1;
    }
    return r;
}

int or_is_prime(uint64_t p) {
    if (p < 2) return 0;
    for (uint64_t d = 2; d * d <= p; ++d)
        if (p % d == 0) return 0;
    return 1;
}

/* Smallest generator of the multiplicative group of Z_p (p prime). */
uint64_t or_primitive_root(uint64_t p) {
    uint64_t m = p - 1, fac[64];
    int nf = 0;
    for (uint64_t d = 2; d * d <= m; ++d) {
        if (m % d == 0) {
            fac[nf++] = d;
            while (m % d == 0) m /= d;
        }
    }
    if (m > 1) fac[nf++] = m;
    for (uint64_t g = 2; g < p; ++g) {
        int ok = 1;
        for (int i = 0; i < nf && ok; ++i)
            if (powmod(g, (p - 1) / fac[i], p) == 1) ok = 0;
        if (ok) return g;
    }
    return 0;
}

/* omega_N (or its inverse): an element of order exactly N, N | p - 1.
 * Returns 0 when N does not divide p - 1. */
uint64_t or_root_of_unity(uint64_t p, uint64_t N, int inverse) {
    if (N == 0 || (p - 1) % N != 0) return 0;
    uint64_t w = powmod(or_primitive_root(p), (p - 1) / N, p);
    return inverse ? powmod(w, p - 2, p) : w;
}

uint64_t or_inverse(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }

/* ------------------------------------------------------- 2D transforms --- */

/* The 2D DFT over Z_p written out as its double sum, O(F^2) per channel:
 * X[k1][k2] = sum_{i1,i2} x[i1][i2] omega_H^{i1 k1} omega_W^{i2 k2} mod p
 * (Eq. (ntt_transform_eq) along both axes). Inverse: omega^-1, times (HW)^-1. */
void or_dft2d_direct(uint64_t p, int64_t batch, int H, int W, const uint32_t *in, uint32_t *out,
                     int inverse) {
    uint64_t wH = or_root_of_unity(p, (uint64_t)H, inverse);
    uint64_t wW = or_root_of_unity(p, (uint64_t)W, inverse);
    uint64_t scale = inverse ? or_inverse((uint64_t)H * (uint64_t)W % p, p) : 1;
    int64_t F = (int64_t)H * W;
    for (int64_t t = 0; t < batch; ++t) {
        const uint32_t *x = in + t * F;
        uint32_t *X = out + t * F;
        for (int k1 = 0; k1 < H; ++k1)
            for (int k2 = 0; k2 < W; ++k2) {
                uint64_t acc = 0;
                for (int i1 = 0; i1 < H; ++i1)
                    for (int i2 = 0; i2 < W; ++i2) {
                        uint64_t tw = mulmod(powmod(wH, (uint64_t)i1 * k1, p),
                                             powmod(wW, (uint64_t)i2 * k2, p), p);
                        acc = (acc + mulmod(x[i1 * W + i2] % p, tw, p)) % p;
                    }
                X[k1 * W + k2] = (uint32_t)mulmod(acc, scale, p);
            }
    }
}

/* The same 2D transform, evaluated axis by axis: a length-W DFT of every row,
 * then a length-H DFT of every column. Each 1D DFT is its plain sum
 * sum_i x_i omega^{ik}, O(L^2). Separable because omega_H^{i1k1} omega_W^{i2k2}
 * factors; no fast algorithm is used. In-place (in == out) is allowed. */
void or_ntt2d(uint64_t p, int64_t batch, int H, int W, const uint32_t *in, uint32_t *out,
              int inverse) {
    uint64_t wH = or_root_of_unity(p, (uint64_t)H, inverse);
    uint64_t wW = or_root_of_unity(p, (uint64_t)W, inverse);
    uint64_t scale = inverse ? or_inverse((uint64_t)H * (uint64_t)W % p, p) : 1;
    int64_t F = (int64_t)H * W;
    uint64_t *powH = malloc(sizeof(uint64_t) * H), *powW = malloc(sizeof(uint64_t) * W);
    for (int e = 0; e < H; ++e) powH[e] = powmod(wH, (uint64_t)e, p);
    for (int e = 0; e < W; ++e) powW[e] = powmod(wW, (uint64_t)e, p);
#pragma omp parallel
    {
        uint64_t *tmp = malloc(sizeof(uint64_t) * F);
#pragma omp for schedule(static)
        for (int64_t t = 0; t < batch; ++t) {
            const uint32_t *x = in + t * F;
            uint32_t *X = out + t * F;
            for (int i1 = 0; i1 < H; ++i1) /* rows */
                for (int k2 = 0; k2 < W; ++k2) {
                    uint64_t acc = 0;
                    for (int i2 = 0; i2 < W; ++i2)
                        acc = (acc + mulmod(x[i1 * W + i2] % p, powW[(int64_t)i2 * k2 % W], p)) % p;
                    tmp[i1 * W + k2] = acc;
                }
            for (int k2 = 0; k2 < W; ++k2) /* columns */
                for (int k1 = 0; k1 < H; ++k1) {
                    uint64_t acc = 0;
                    for (int i1 = 0; i1 < H; ++i1)
                        acc = (acc + mulmod(tmp[i1 * W + k2], powH[(int64_t)i1 * k1 % H], p)) % p;
                    X[k1 * W + k2] = (uint32_t)mulmod(acc, scale, p);
                }
        }
        free(tmp);
    }
    free(powH);
    free(powW);
}

/* Server setup: each filter w[o][i] (kh x kw signed ints) reduced mod p,
 * zero-padded into the top-left of the H x W grid, then transformed
 * (Sec. 4.1, "Line 3-4": pad, DFT2D and flatten of the weight matrix). */
void or_weight_prep(uint64_t p, int Cout, int Cin, int kh, int kw, int H, int W, const int32_t *w,
                    uint32_t *w_hat) {
    int64_t F = (int64_t)H * W, nt = (int64_t)Cout * Cin;
    memset(w_hat, 0, sizeof(uint32_t) * (size_t)(nt * F));
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < kh; ++a)
            for (int b = 0; b < kw; ++b) {
                int64_t v = w[(t * kh + a) * kw + b] % (int64_t)p;
                if (v < 0) v += (int64_t)p;
                w_hat[t * F + a * W + b] = (uint32_t)v;
            }
    or_ntt2d(p, nt, H, W, w_hat, w_hat, 0);
}

/* Direct cyclic convolution summed over input channels (Eq. (f_conv) read
 * in the spatial domain; the channel sum of a conv layer):
 * y[b][o][m1][m2] = sum_i sum_{j1<kh, j2<kw} w[o][i][j1][j2]
 *                   * x[b][i][(m1-j1) mod H][(m2-j2) mod W]   mod p. */
void or_cyclic_conv(uint64_t p, int B, int Cin, int Cout, int H, int W, int kh, int kw,
                    const uint32_t *x, const int32_t *w, uint32_t *y) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < Cout; ++o)
            for (int m1 = 0; m1 < H; ++m1)
                for (int m2 = 0; m2 < W; ++m2) {
                    uint64_t acc = 0;
                    for (int i = 0; i < Cin; ++i)
                        for (int j1 = 0; j1 < kh; ++j1)
                            for (int j2 = 0; j2 < kw; ++j2) {
                                int64_t wv = w[(((int64_t)o * Cin + i) * kh + j1) * kw + j2] % (int64_t)p;
                                if (wv < 0) wv += (int64_t)p;
                                int r1 = ((m1 - j1) % H + H) % H, r2 = ((m2 - j2) % W + W) % W;
                                uint64_t xv = x[(((int64_t)b * Cin + i) * H + r1) * W + r2] % p;
                                acc = (acc + mulmod((uint64_t)wv, xv, p)) % p;
                            }
                    y[(((int64_t)b * Cout + o) * H + m1) * W + m2] = (uint32_t)acc;
                }
}

/* -------------------------------------------------- a-vector generator --- */

#define SM64_GAMMA 0x9e3779b97f4a7c15ULL

/* Output number k (k >= 1) of SplitMix64 seeded with `seed`: the state after
 * k increments by the golden-ratio gamma, passed through the published
 * 64-bit finaliser (xor-shift 30, multiply, xor-shift 27, multiply,
 * xor-shift 31). */
uint64_t or_splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * SM64_GAMMA;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* --------------------------------------------------------------- LWE --- */

uint64_t or_delta(uint64_t p) { return (uint64_t)((((u128)1) << 64) / p); }

/* Enc of the B*C*F plaintexts m[b][c][f] in [0,p) under ternary key s
 * (Eq. (bfv_enc), one coefficient per ciphertext), e[b][c][f] the errors.
 * ct is [B][F][n+1][C]: ciphertext (b, c, f) has word j at ct[b][f][j][c]. */
void or_encrypt(uint64_t p, int64_t B, int C, int64_t F, int n, const uint32_t *m, const int8_t *s,
                const int32_t *e, uint64_t seed_a, uint64_t ct_index0, uint64_t *ct) {
    uint64_t delta = or_delta(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t f = 0; f < F; ++f)
            for (int c = 0; c < C; ++c) {
                uint64_t q = (uint64_t)((b * F + f) * C + c), dot = 0;
                uint64_t *w = ct + (b * F + f) * (int64_t)(n + 1) * C + c; /* word j at w[j * C] */
                for (int j = 0; j < n; ++j) {
                    uint64_t a = or_splitmix64(seed_a, (ct_index0 + q) * (uint64_t)n + (uint64_t)j + 1);
                    w[(int64_t)j * C] = a;
                    if (s[j] == 1) dot += a;
                    else if (s[j] == -1) dot -= a;
                }
                int64_t mi = (b * C + c) * F + f;
                w[(int64_t)n * C] = dot + (uint64_t)(int64_t)e[mi] + delta * (uint64_t)m[mi];
            }
}

/* Decryption phase phi = b - <a, s> mod 2^64 of one ciphertext whose word j
 * is at w[j * stride]. */
uint64_t or_phase(int n, const uint64_t *w, int64_t stride, const int8_t *s) {
    uint64_t dot = 0;
    for (int j = 0; j < n; ++j) {
        if (s[j] == 1) dot += w[j * stride];
        else if (s[j] == -1) dot -= w[j * stride];
    }
    return w[(int64_t)n * stride] - dot;
}

/* Dec of ct [B][F][n+1][C] into m[b][c][f]:
 * m = floor((phi * p + 2^63) / 2^64) mod p, in exact 128-bit arithmetic. */
void or_decrypt(uint64_t p, int64_t B, int C, int64_t F, int n, const uint64_t *ct, const int8_t *s,
                uint32_t *m) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t f = 0; f < F; ++f)
            for (int c = 0; c < C; ++c) {
                uint64_t phi = or_phase(n, ct + (b * F + f) * (int64_t)(n + 1) * C + c, C, s);
                u128 t = (u128)phi * p + (((u128)1) << 63);
                uint64_t v = (uint64_t)(t >> 64);
                m[(b * C + c) * F + f] = (uint32_t)(v % p);
            }
}

/* A seeded ciphertext: Sec. 5.1 notes that the public constants of a
 * ciphertext can be generated offline. Here they are the a-words of the
 * SplitMix64 stream above, so a batch of ciphertexts is fully given by seed_a,
 * its first index and its b words, and only the b words travel. Expands
 * bw[b][f][c] into ct [B][F][n+1][C]: word j < n of ciphertext
 * q = (b F + f) C + c is output number (q0 + q) n + j + 1 of the generator
 * seeded with seed_a (the words or_encrypt writes), word n is bw[b][f][c]. */
void or_expand_seeded(int64_t B, int C, int64_t F, int n, uint64_t seed_a, uint64_t ct_index0, const uint64_t *bw,
                      uint64_t *ct) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t f = 0; f < F; ++f)
            for (int c = 0; c < C; ++c) {
                uint64_t q = (uint64_t)((b * F + f) * C + c);
                uint64_t *w = ct + (b * F + f) * (int64_t)(n + 1) * C + c;
                for (int j = 0; j < n; ++j)
                    w[(int64_t)j * C] = or_splitmix64(seed_a, (ct_index0 + q) * (uint64_t)n + (uint64_t)j + 1);
                w[(int64_t)n * C] = bw[(b * F + f) * C + c];
            }
}

/* Rounded-Gaussian errors drawn from the public generator (the on-device
 * sampler's definition; the LWE error distribution of Sec. 3.1 with the
 * sigma = 3.2 of the design notes). T holds K cumulative thresholds of |e| on
 * a 2^48 grid, T[k] = floor(2^48 P(|e| <= k)); the error of ciphertext
 * q = (b F + f) C + c comes from output number ct_index0 + q + 1 of the
 * generator seeded with seed_e: its top bit is the sign, bits 15..62 a
 * uniform v < 2^48, and |e| is the number of thresholds <= v. e is stored
 * like the plaintexts, e[(b C + c) F + f]. */
void or_sample_errors(const uint64_t *T, int K, uint64_t seed_e, uint64_t ct_index0, int64_t B, int C, int64_t F,
                      int32_t *e) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t f = 0; f < F; ++f)
            for (int c = 0; c < C; ++c) {
                uint64_t q = (uint64_t)((b * F + f) * C + c);
                uint64_t u = or_splitmix64(seed_e, ct_index0 + q + 1);
                uint64_t v = (u >> 15) & ((1ULL << 48) - 1);
                int mag = 0;
                for (int k = 0; k < K; ++k)
                    if (T[k] <= v) ++mag;
                e[(b * C + c) * F + f] = (u >> 63) && mag ? -mag : mag;
            }
}

/* --------------------------------------------------------- HomConv --- */

/* One output ciphertext of HomConv for (image b, output channel o,
 * frequency f): sum_i W^[o,i,f] * ct_in(b, i, f) mod 2^64 word by word, then
 * + Delta * r[b,o,f] on the b word. ct_in [B][F][n+1][Cin],
 * w_hat [Cout][Cin][F] (integers in [0,p)), r [B][Cout][F]; the result's
 * word j goes to out[j * ostride]. */
static void homconv_one(uint64_t p, int Cin, int Cout, int64_t F, int n, const uint64_t *ct_in,
                        const uint32_t *w_hat, const uint32_t *r, int64_t b, int64_t o, int64_t f,
                        uint64_t *out, int64_t ostride) {
    const uint64_t *blk = ct_in + (b * F + f) * (int64_t)(n + 1) * Cin;
    for (int j = 0; j <= n; ++j) {
        uint64_t acc = 0;
        for (int i = 0; i < Cin; ++i)
            acc += (uint64_t)w_hat[(o * Cin + i) * F + f] * blk[(int64_t)j * Cin + i];
        out[j * ostride] = acc;
    }
    out[n * ostride] += or_delta(p) * (uint64_t)r[(b * Cout + o) * F + f];
}

void or_homconv(uint64_t p, int B, int Cin, int Cout, int64_t F, int n, const uint64_t *ct_in,
                const uint32_t *w_hat, const uint32_t *r, uint64_t *ct_out) {
#pragma omp parallel for collapse(3) schedule(static)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t f = 0; f < F; ++f)
            for (int64_t o = 0; o < Cout; ++o)
                homconv_one(p, Cin, Cout, F, n, ct_in, w_hat, r, b, o, f,
                            ct_out + (b * F + f) * (int64_t)(n + 1) * Cout + o, Cout);
}

/* HomConv restricted to the listed outputs: sel holds nsel triples
 * (b, o, f); out is [nsel][n+1] (one ciphertext's words per row). */
void or_homconv_select(uint64_t p, int B, int Cin, int Cout, int64_t F, int n, const uint64_t *ct_in,
                       const uint32_t *w_hat, const uint32_t *r, int64_t nsel, const int64_t *sel,
                       uint64_t *out) {
    (void)B;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nsel; ++k)
        homconv_one(p, Cin, Cout, F, n, ct_in, w_hat, r, sel[3 * k], sel[3 * k + 1], sel[3 * k + 2],
                    out + k * (int64_t)(n + 1), 1);
}

/* The server's spatial share s_B = INTT2D(-r mod p) (Sec. 4.1, "Line 4-6"). */
void or_server_share(uint64_t p, int64_t batch, int H, int W, const uint32_t *r, uint32_t *s_b) {
    int64_t F = (int64_t)H * W;
    for (int64_t k = 0; k < batch * F; ++k) s_b[k] = (uint32_t)((p - r[k] % p) % p);
    or_ntt2d(p, batch, H, W, s_b, s_b, 1);
}

/* ------------------------------------------------- chained rounds --- */

/* HomRec (Eq. (homrec); Fig. 2's re-entry of the server's share, Eq. (dft_convolution0)): the
 * server adds its transformed share to the client's ciphertexts as a
 * plaintext, [s_A] (+) s_B = [s_A + s_B mod p]: Delta * s_hat[b][c][f] is
 * added to the b word of ciphertext (b, c, f) of ct [B][F][n+1][C], in place.
 * (Delta p = 2^64 - 1, so a sum that wraps past p costs -1 of noise.) */
void or_homrec(uint64_t p, int64_t B, int C, int64_t F, int n, uint64_t *ct, const uint32_t *s_hat) {
    const uint64_t delta = or_delta(p);
    for (int64_t b = 0; b < B; ++b)
        for (int64_t f = 0; f < F; ++f)
            for (int c = 0; c < C; ++c)
                ct[((b * F + f) * (int64_t)(n + 1) + n) * C + c] += delta * (uint64_t)s_hat[(b * C + c) * F + f];
}

/* Stand-in for the oblivious activation between the rounds of Fig. 2, computed in the
 * clear: y = s_A + s_B mod p, u = f(y) (act 0: identity, 1: square mod p),
 * and the client's next share s_A' = u - s_B' mod p for the server's fresh
 * share s_B'. All arrays hold count residues in [0, p). */
void or_reshare(uint64_t p, int64_t count, const uint32_t *s_a, const uint32_t *s_b, const uint32_t *s_b_next,
                int act, uint32_t *s_a_next) {
    for (int64_t k = 0; k < count; ++k) {
        uint64_t y = ((uint64_t)s_a[k] + s_b[k]) % p;
        uint64_t u = act == 1 ? mulmod(y, y, p) : y;
        s_a_next[k] = (uint32_t)((u + p - s_b_next[k]) % p);
    }
}

/* ------------------------------------------------------------ threads --- */
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sets the OpenMP thread count used by the loops above (k <= 0 keeps it);
 * returns the count now in effect (1 when built without OpenMP). */
int or_set_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
    return omp_get_max_threads();
#else
    (void)k;
    return 1;
#endif
}
