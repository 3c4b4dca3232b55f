/*
 * Host driver that runs every function of the CPU oracle (oracle/ensei_oracle.c)
 * once on small inputs with a few self-checks, so that the oracle can be built
 * and run under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py). Exits non-zero on a failed check; the
 * sanitizers abort on their own findings.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_is_prime(uint64_t p);
uint64_t or_primitive_root(uint64_t p);
uint64_t or_root_of_unity(uint64_t p, uint64_t N, int inverse);
uint64_t or_inverse(uint64_t a, uint64_t p);
void or_dft2d_direct(uint64_t p, int64_t batch, int H, int W, const uint32_t *in, uint32_t *out, int inverse);
void or_ntt2d(uint64_t p, int64_t batch, int H, int W, const uint32_t *in, uint32_t *out, int inverse);
void or_weight_prep(uint64_t p, int Cout, int Cin, int kh, int kw, int H, int W, const int32_t *w, uint32_t *w_hat);
void or_cyclic_conv(uint64_t p, int B, int Cin, int Cout, int H, int W, int kh, int kw, const uint32_t *x,
                    const int32_t *w, uint32_t *y);
uint64_t or_splitmix64(uint64_t seed, uint64_t k);
uint64_t or_delta(uint64_t p);
void or_encrypt(uint64_t p, int64_t B, int C, int64_t F, int n, const uint32_t *m, const int8_t *s, const int32_t *e,
                uint64_t seed_a, uint64_t ct_index0, uint64_t *ct);
uint64_t or_phase(int n, const uint64_t *w, int64_t stride, const int8_t *s);
void or_decrypt(uint64_t p, int64_t B, int C, int64_t F, int n, const uint64_t *ct, const int8_t *s, uint32_t *m);
void or_expand_seeded(int64_t B, int C, int64_t F, int n, uint64_t seed_a, uint64_t ct_index0, const uint64_t *bw,
                      uint64_t *ct);
void or_sample_errors(const uint64_t *T, int K, uint64_t seed_e, uint64_t ct_index0, int64_t B, int C, int64_t F,
                      int32_t *e);
void or_homconv(uint64_t p, int B, int Cin, int Cout, int64_t F, int n, const uint64_t *ct_in, const uint32_t *w_hat,
                const uint32_t *r, uint64_t *ct_out);
void or_homconv_select(uint64_t p, int B, int Cin, int Cout, int64_t F, int n, const uint64_t *ct_in,
                       const uint32_t *w_hat, const uint32_t *r, int64_t nsel, const int64_t *sel, uint64_t *out);
void or_server_share(uint64_t p, int64_t batch, int H, int W, const uint32_t *r, uint32_t *s_b);
void or_homrec(uint64_t p, int64_t B, int C, int64_t F, int n, uint64_t *ct, const uint32_t *s_hat);
void or_reshare(uint64_t p, int64_t count, const uint32_t *s_a, const uint32_t *s_b, const uint32_t *s_b_next, int act,
                uint32_t *s_a_next);
int or_set_threads(int k);

static int failures = 0;
#define CHECK(cond)                                              \
    do {                                                         \
        if (!(cond)) {                                           \
            printf("FAILED line %d: %s\n", __LINE__, #cond);     \
            ++failures;                                          \
        }                                                        \
    } while (0)

static uint64_t rng = 0x1234567u;
static uint64_t next_u64(void) {
    rng += 0x9e3779b97f4a7c15ULL;
    uint64_t z = rng;
    z = (z ^ (z >> 31)) * 0x7fb5d329728ea185ULL;
    return z ^ (z >> 29);
}

int main(void) {
    const uint64_t p = 65537;
    enum { B = 2, Cin = 3, Cout = 2, H = 8, W = 4, F = H * W, kh = 3, kw = 2, n = 16 };
    or_set_threads(2);
    CHECK(or_is_prime(p) && !or_is_prime(65535));
    CHECK(or_primitive_root(p) == 3);
    CHECK(or_inverse(or_root_of_unity(p, 8, 0), p) == or_root_of_unity(p, 8, 1));

    uint32_t *x = malloc(sizeof(uint32_t) * B * Cin * F), *xh = malloc(sizeof(uint32_t) * B * Cin * F);
    uint32_t *xd = malloc(sizeof(uint32_t) * B * Cin * F), *back = malloc(sizeof(uint32_t) * B * Cin * F);
    for (int k = 0; k < B * Cin * F; ++k) x[k] = (uint32_t)(next_u64() % 256);
    or_ntt2d(p, B * Cin, H, W, x, xh, 0);
    or_dft2d_direct(p, B * Cin, H, W, x, xd, 0);
    CHECK(memcmp(xh, xd, sizeof(uint32_t) * B * Cin * F) == 0);
    or_ntt2d(p, B * Cin, H, W, xh, back, 1);
    CHECK(memcmp(back, x, sizeof(uint32_t) * B * Cin * F) == 0);

    int32_t *w = malloc(sizeof(int32_t) * Cout * Cin * kh * kw);
    for (int k = 0; k < Cout * Cin * kh * kw; ++k) w[k] = (int32_t)(next_u64() % 17) - 8;
    uint32_t *wh = malloc(sizeof(uint32_t) * Cout * Cin * F), *y = malloc(sizeof(uint32_t) * B * Cout * F);
    or_weight_prep(p, Cout, Cin, kh, kw, H, W, w, wh);
    or_cyclic_conv(p, B, Cin, Cout, H, W, kh, kw, x, w, y);

    int8_t s[n];
    for (int j = 0; j < n; ++j) s[j] = (int8_t)((int)(next_u64() % 3) - 1);
    uint64_t T[32];
    for (int k = 0; k < 32; ++k) T[k] = (1ULL << 48) - (1ULL << (47 - k));
    int32_t *e = malloc(sizeof(int32_t) * B * Cin * F);
    or_sample_errors(T, 32, 99, 0, B, Cin, F, e);
    uint64_t *ct = malloc(sizeof(uint64_t) * B * F * (n + 1) * Cin);
    or_encrypt(p, B, Cin, F, n, xh, s, e, 7, 0, ct);
    uint32_t *m = malloc(sizeof(uint32_t) * B * Cin * F);
    or_decrypt(p, B, Cin, F, n, ct, s, m);
    CHECK(memcmp(m, xh, sizeof(uint32_t) * B * Cin * F) == 0);
    (void)or_phase(n, ct, Cin, s);

    uint64_t *bw = malloc(sizeof(uint64_t) * B * F * Cin), *ct2 = malloc(sizeof(uint64_t) * B * F * (n + 1) * Cin);
    for (int b = 0; b < B; ++b)
        for (int f = 0; f < F; ++f)
            for (int c = 0; c < Cin; ++c) bw[(b * F + f) * Cin + c] = ct[((b * F + f) * (n + 1) + n) * Cin + c];
    or_expand_seeded(B, Cin, F, n, 7, 0, bw, ct2);
    CHECK(memcmp(ct, ct2, sizeof(uint64_t) * B * F * (n + 1) * Cin) == 0);

    uint32_t *r = malloc(sizeof(uint32_t) * B * Cout * F);
    for (int k = 0; k < B * Cout * F; ++k) r[k] = (uint32_t)(next_u64() % p);
    uint64_t *out = malloc(sizeof(uint64_t) * B * F * (n + 1) * Cout);
    or_homconv(p, B, Cin, Cout, F, n, ct, wh, r, out);
    int64_t sel[3] = {1, 1, F - 1};
    uint64_t one[n + 1];
    or_homconv_select(p, B, Cin, Cout, F, n, ct, wh, r, 1, sel, one);
    for (int j = 0; j <= n; ++j) CHECK(one[j] == out[((1 * F + F - 1) * (n + 1) + j) * Cout + 1]);

    uint32_t *mo = malloc(sizeof(uint32_t) * B * Cout * F), *sa = malloc(sizeof(uint32_t) * B * Cout * F);
    uint32_t *sb = malloc(sizeof(uint32_t) * B * Cout * F);
    or_decrypt(p, B, Cout, F, n, out, s, mo);
    or_ntt2d(p, B * Cout, H, W, mo, sa, 1);
    or_server_share(p, B * Cout, H, W, r, sb);
    for (int k = 0; k < B * Cout * F; ++k) CHECK((sa[k] + sb[k]) % p == y[k]);

    uint32_t *sbn = malloc(sizeof(uint32_t) * B * Cout * F), *san = malloc(sizeof(uint32_t) * B * Cout * F);
    for (int k = 0; k < B * Cout * F; ++k) sbn[k] = (uint32_t)(next_u64() % p);
    or_reshare(p, B * Cout * F, sa, sb, sbn, 1, san);
    for (int k = 0; k < B * Cout * F; ++k) CHECK((san[k] + sbn[k]) % p == (uint64_t)y[k] * y[k] % p);
    or_homrec(p, B, Cin, F, n, ct, xh);
    or_decrypt(p, B, Cin, F, n, ct, s, m);
    for (int k = 0; k < B * Cin * F; ++k) CHECK(m[k] == (2 * (uint64_t)xh[k]) % p);
    (void)or_splitmix64(1, 1);
    (void)or_delta(p);

    free(x), free(xh), free(xd), free(back), free(w), free(wh), free(y), free(e), free(ct), free(m), free(bw);
    free(ct2), free(r), free(out), free(mo), free(sa), free(sb), free(sbn), free(san);
    printf("%s\n", failures ? "oracle driver FAILED" : "oracle driver ok");
    return failures ? 1 : 0;
}
