"""Pins for the packed (BFV / RLWE) oracle (oracle/bfv.py): checks against
what the paper and the mathematics fix, never against the oracle itself.

Each ``check_*`` takes a ``BfvOracle`` and raises AssertionError on a
disagreement with: Table 2's printed moduli and bit lengths, brute-force
searches and closed forms in Python integers, schoolbook negacyclic products
(numpy integer convolutions), a big-integer SplitMix64, Python big-integer
CRT and Delta, and the exact noise identity of a plaintext-ciphertext product
derived from Delta t = q - rho. ``tests/test_bfv_oracle.py`` runs them;
``tests/test_bfv_mutants.py`` plants mistakes in copies of the C oracle.
"""
from __future__ import annotations

import os

import numpy as np

from oracle import bfv
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
L = 2
# a toy set for the heavier structural checks (same rules, n = 64): t = 257
# and the High set's limbs, all primes = 1 mod 128
TOY = bfv.Params("toy", 257, 1073692673, 561770497, 64)


def _rng(seed):
    return np.random.default_rng(seed)


def _delta(pr) -> int:
    """Delta: the integer nearest to q / t (exact rationals)."""
    from fractions import Fraction

    return int(Fraction(pr.q, pr.t) + Fraction(1, 2))


def _sets():
    return list(bfv.table2_params().values())


def _table2_printed():
    """name -> (p_E, ceil(lg q), n) as printed in Table 2."""
    out = {}
    for line in open(os.path.join(GOLDEN, "table2_moduli.txt")):
        f = line.split("#", 1)[0].split()
        if len(f) == 5:
            out[f[0].lower()] = (int(f[2]), int(f[3]), int(f[4]))
    return out


def _is_prime(m: int) -> bool:
    return m > 1 and all(m % d for d in range(2, int(m**0.5) + 1))


def _smallest_generator(m: int) -> int:
    """Smallest primitive root of the prime m, by factoring m - 1 (trial division)."""
    r, fac, d = m - 1, [], 2
    while d * d <= r:
        if r % d == 0:
            fac.append(d)
            while r % d == 0:
                r //= d
        d += 1
    if r > 1:
        fac.append(r)
    return next(g for g in range(2, m) if all(pow(g, (m - 1) // f, m) != 1 for f in fac))


def negacyclic_product(a, b, m: int) -> np.ndarray:
    """a * b in Z_m[X]/(X^n + 1) by schoolbook convolution (numpy integer
    convolve; b split into 12-bit pieces so that no partial sum overflows)."""
    a = np.asarray(a, dtype=np.int64) % m
    b = np.asarray(b, dtype=np.int64) % m
    n = a.size
    acc = np.zeros(2 * n - 1, dtype=object)
    shift = 0
    while b.any():
        piece = b & 0xFFF
        c = np.convolve(a, piece)  # each term < 2^31 * 2^12, n of them < 2^54
        acc = acc + (c.astype(object) % m) * (1 << shift)
        b = b >> 12
        shift += 12
    full = [int(x) % m for x in acc] + [0]
    return np.array([(full[k] - full[k + n]) % m for k in range(n)], dtype=np.int64)


def negacyclic_product_z(a, b) -> list:
    """a * b in Z[X]/(X^n + 1) for small signed integer vectors (exact: object dtype)."""
    a = np.asarray(a, dtype=object)
    b = np.asarray(b, dtype=object)
    n = a.size
    c = np.convolve(a, b)
    c = list(c) + [0]
    return [c[k] - c[k + n] for k in range(n)]


# ------------------------------------------------------------- moduli ---


def check_params_against_table2(orc):
    printed = _table2_printed()
    for pr in _sets():
        p_e, lgq, n = printed[pr.name]
        assert (pr.t, pr.n) == (p_e, n)
        assert (pr.q0 * pr.q1 - 1).bit_length() == lgq and 2 ** (lgq - 1) < pr.q <= 2**lgq  # ceil(lg q)
        for m in (pr.t, pr.q0, pr.q1):
            assert _is_prime(m) and orc.is_prime(m)
            assert (m - 1) % (2 * n) == 0  # X^n + 1 splits: 2n-th roots exist
        assert pr.q0 != pr.q1


def check_psi(orc):
    for pr in _sets() + [TOY]:
        for m in (pr.t, pr.q0, pr.q1):
            psi = orc.psi(m, pr.n)
            assert pow(psi, pr.n, m) == m - 1  # psi^n = -1: order exactly 2n
            assert psi == pow(_smallest_generator(m), (m - 1) // (2 * pr.n), m)
    for m, n in ((17, 4), (97, 8), (257, 16)):
        assert orc.psi(m, n) == bf.brute_root(m, 2 * n)
    assert orc.psi(12289, 4096) == 0  # 2n = 8192 does not divide 12288


# ---------------------------------------------------------- transforms ---


def check_negacyclic_definition(orc):
    """Small sizes against the sum written out in Python integers, and the
    transform of the monomials X^j (closed form psi^((2k+1) j))."""
    g = _rng(1)
    for m, n in ((17, 4), (97, 8), (257, 16), (7681, 64)):
        psi = bf.brute_root(m, 2 * n)
        x = g.integers(0, m, size=(3, n))
        got = orc.negacyclic(x, m)
        for t in range(3):
            for k in range(n):
                assert got[t, k] == sum(int(x[t, j]) * pow(psi, (2 * k + 1) * j, m) for j in range(n)) % m
        inv = orc.negacyclic(got, m, inverse=True)
        assert np.array_equal(inv, x)
        for j in (0, 1, n - 1):
            e = np.zeros(n, dtype=np.int64)
            e[j] = 1
            assert [int(v) for v in orc.negacyclic(e, m)] == [pow(psi, (2 * k + 1) * j, m) for k in range(n)]


def check_convolution_theorem(orc):
    """Slot-wise products are negacyclic products of coefficients, at n = 2048
    for every modulus of Table 2, against schoolbook multiplication."""
    g = _rng(2)
    for pr in _sets():
        for m in (pr.t, pr.q0, pr.q1):
            a = g.integers(0, m, size=pr.n)
            b = g.integers(0, m, size=pr.n)
            A, Bv = orc.negacyclic(a, m).astype(np.int64), orc.negacyclic(b, m).astype(np.int64)
            prod = np.array([int(x) * int(y) % m for x, y in zip(A, Bv)], dtype=np.int64)
            assert np.array_equal(prod, orc.negacyclic(negacyclic_product(a, b, m), m).astype(np.int64))
            assert np.array_equal(orc.negacyclic(A, m, inverse=True).astype(np.int64), a)


# ------------------------------------------------------------- Enc/Dec ---


def _crt(r0, r1, q0, q1) -> list:
    """x mod q0 q1 from residues, by Python big integers (search-free formula check below)."""
    out = []
    for a, b in zip(r0, r1):
        x = (int(a) * q1 * pow(q1, -1, q0) + int(b) * q0 * pow(q0, -1, q1)) % (q0 * q1)
        out.append(x)
    return out


def check_enc_phase_exact(orc):
    """INTT_q(b^ - a^ . s^) = Delta u + e exactly (mod q), u = INTT_t(v): the
    LWE form of Eq. (bfv_enc) in the ring; phases joined by CRT."""
    g = _rng(3)
    for pr in _sets() + [TOY]:
        v = g.integers(0, pr.t, size=(2, pr.n))
        v[0, :4] = [0, pr.t - 1, 1, pr.t // 2]
        s = g.integers(-1, 2, size=pr.n).astype(np.int8)
        e = np.rint(g.normal(0, 4.0, size=v.shape)).astype(np.int32)
        ct = orc.encrypt(pr, v, s, e, seed_a=11)
        phi = orc.phase(pr, ct, s)
        u = orc.negacyclic(v, pr.t, inverse=True)
        # the phase independently: b^ - a^ s^ per limb with s^ = NTT(s), inverse, CRT
        for i in range(2):
            res = []
            for l, m in enumerate((pr.q0, pr.q1)):
                s_hat = orc.negacyclic(np.where(s < 0, m - 1, s.astype(np.int64)), m).astype(object)
                a, b = ct[i, l, 0].astype(object), ct[i, l, 1].astype(object)
                res.append(orc.negacyclic(np.array([(bb - aa * ss) % m for aa, bb, ss in zip(a, b, s_hat)],
                                                   dtype=np.int64), m, inverse=True))
            want = [(_delta(pr) * int(uu) + int(ee)) % pr.q for uu, ee in zip(u[i], e[i])]
            assert _crt(res[0], res[1], pr.q0, pr.q1) == want
            assert [int(x) for x in phi[i]] == want


def check_roundtrip(orc):
    """Dec(Enc(v)) = v for random and edge slot values, every parameter set."""
    g = _rng(4)
    for pr in _sets():
        v = g.integers(0, pr.t, size=(2, pr.n))
        v[1] = pr.t - 1
        v[1, ::3] = 0
        s = g.integers(-1, 2, size=pr.n).astype(np.int8)
        e = np.rint(g.normal(0, 4.0, size=v.shape)).astype(np.int32)
        assert np.array_equal(orc.decrypt(pr, orc.encrypt(pr, v, s, e, seed_a=5, ct_index0=7), s), v)


def check_decryption_rounding(orc):
    """m = round(t phi / q) with ties impossible (q odd): the decoded
    coefficients of trivial ciphertexts (a^ = 0) at phases just inside and
    just outside Delta/2 of a multiple of Delta, against exact rationals."""
    from fractions import Fraction

    pr = TOY
    s = np.zeros(pr.n, dtype=np.int8)
    g = _rng(5)
    phis = [0, _delta(pr) // 2, _delta(pr) // 2 + 1, pr.q - 1, pr.q - _delta(pr) // 2 - 1, 3 * _delta(pr) + _delta(pr) // 2]
    phis += [int(x) for x in g.integers(0, pr.q, size=pr.n - len(phis))]
    ct = np.zeros((L, 2, pr.n), dtype=np.uint32)
    for l, m in enumerate((pr.q0, pr.q1)):
        ct[l, 1] = orc.negacyclic(np.array([x % m for x in phis], dtype=np.int64), m)
    got = orc.negacyclic(orc.decrypt(pr, ct, s), pr.t, inverse=True)  # back to coefficients
    for x, m in zip(phis, got):
        r = Fraction(pr.t * x, pr.q)
        assert int(m) == int(r + Fraction(1, 2)) % pr.t


def check_public_constants(orc):
    """a^ words: limb l, slot k of ciphertext c0 + i is SplitMix64 output
    ((c0 + i) L + l) n + k + 1 of seed_a, mod q_l (big-integer generator)."""
    pr = TOY
    g = _rng(6)
    v = g.integers(0, pr.t, size=(2, pr.n))
    s = g.integers(-1, 2, size=pr.n).astype(np.int8)
    ct = orc.encrypt(pr, v, s, np.zeros(v.shape, np.int32), seed_a=99, ct_index0=3)
    stream = bf.splitmix64_stream(99, (3 + 2) * L * pr.n + 1)
    for i in range(2):
        for l, m in enumerate((pr.q0, pr.q1)):
            base = ((3 + i) * L + l) * pr.n
            assert [int(x) for x in ct[i, l, 0]] == [stream[base + k] % m for k in range(pr.n)]


# ------------------------------------------------------------- packing ---


def check_pack_and_fold(orc):
    """Channel g P + j of the spectra lands in slots [j F, (j+1) F) of vector
    g (F <= n), or frequency chunk k in vector k (F > n); folding adds the P
    blocks."""
    g = _rng(7)
    n = 64
    for C_, F in ((5, 16), (3, 64), (2, 256)):
        x = g.integers(0, 257, size=(2, C_, F))
        v = orc.pack(x, n)
        P, K, G = bfv.shape_counts(C_, F, n)
        assert v.shape == (2, G * K, n)
        want = np.zeros((2, G * K, n), dtype=np.int64)
        for b in range(2):
            for c in range(C_):
                for f in range(F):
                    want[b, (c // P) * K + f // min(F, n), (c % P) * min(F, n) + f % min(F, n)] = x[b, c, f]
        assert np.array_equal(v, want)
        y = orc.fold(TOY, v, F) if K == 1 and G == 1 else None
        if y is not None:
            assert np.array_equal(y[:, 0], x.sum(axis=1) % TOY.t)
    vv = g.integers(0, 257, size=(1, 4, n))  # Cout = 4 outputs, F = 16: 4 blocks each
    assert np.array_equal(orc.fold(TOY, vv, 16), vv.reshape(1, 4, 4, 16).sum(axis=2) % 257)
    vv = g.integers(0, 257, size=(1, 6, n))  # Cout = 3, F = 128 > n: 2 chunks, no blocks
    assert np.array_equal(orc.fold(TOY, vv, 128), vv.reshape(1, 3, 128))


# ----------------------------------------------------- SIMDScMult + share ---


def _conv_case(orc, pr, B, Cin, Cout, F, seed):
    g = _rng(seed)
    P, K, G = bfv.shape_counts(Cin, F, pr.n)
    x_hat = g.integers(0, pr.t, size=(B, Cin, F))
    w_hat = g.integers(0, pr.t, size=(Cout, Cin, F))
    r = g.integers(0, pr.t, size=(B, Cout * K, pr.n))
    s = g.integers(-1, 2, size=pr.n).astype(np.int8)
    e = np.rint(g.normal(0, 4.0, size=(B, G * K, pr.n))).astype(np.int32)
    return x_hat, w_hat, r, s, e, orc.secure_conv(pr, x_hat, w_hat, r, s, e, seed_a=seed)


def check_secure_conv_plaintext(orc):
    """Dec(HomConv(Enc(pack(x^)))) folded = sum_i W^ x^ + fold(r) mod t:
    SIMDScMult, the channel sum and HomShare on packed ciphertexts, for
    several channels per vector (with a partial last vector), one channel
    per vector, and channels spanning two vectors."""
    cases = [(TOY, 2, 10, 3, 16), (TOY, 1, 3, 2, 64), (TOY, 1, 2, 2, 128), (_sets()[0], 1, 3, 2, 1024)]
    for k, (pr, B, Cin, Cout, F) in enumerate(cases):
        x_hat, w_hat, r, s, e, res = _conv_case(orc, pr, B, Cin, Cout, F, 20 + k)
        want = (np.einsum("oif,bif->bof", w_hat.astype(np.int64), x_hat.astype(np.int64)) + res["r_fold"]) % pr.t
        assert np.array_equal(res["y"].astype(np.int64), want), (pr.name, Cin, F)
        # the fold of the masks is the sum of their slot blocks
        P, K, G = bfv.shape_counts(Cin, F, pr.n)
        Fp = min(F, pr.n)
        rf = r.reshape(B, Cout, K, pr.n // Fp, Fp).sum(axis=3).reshape(B, Cout, K * Fp) % pr.t
        assert np.array_equal(res["r_fold"].astype(np.int64), rf)


def check_homconv_noise_identity(orc):
    """The exact phase of an output ciphertext. With w_g the centred lift of
    INTT_t of filter vector g, u_g = INTT_t(v_g) and u_r = INTT_t(r) in
    [0, t), and M = sum_g w_g u_g + u_r in Z[X]/(X^n+1):
        phi_out = Delta [M]_t + (sum_g w_g e_g - rho floor(M / t))  (mod q)
    since Delta t = q - rho (rho = q - Delta t, small and of either sign).
    Checked coefficient by coefficient."""
    pr = TOY
    x_hat, w_hat, r, s, e, res = _conv_case(orc, pr, 1, 10, 2, 16, 40)
    P, K, G = bfv.shape_counts(10, 16, pr.n)
    phi = orc.phase(pr, res["ct_out"], s)
    u = orc.negacyclic(res["v_in"], pr.t, inverse=True).astype(np.int64)
    ur = orc.negacyclic(r, pr.t, inverse=True).astype(np.int64)
    # filter slot vectors by the packing rule, independently of the oracle's
    wv = np.zeros((2, G, pr.n), dtype=np.int64)
    for o in range(2):
        for c in range(10):
            wv[o, c // P, (c % P) * 16:(c % P) * 16 + 16] = w_hat[o, c]
    wc = orc.negacyclic(wv, pr.t, inverse=True).astype(np.int64)
    wc = np.where(wc > pr.t // 2, wc - pr.t, wc)  # centred
    rq = pr.q - _delta(pr) * pr.t
    for o in range(2):
        M = np.array(ur[0, o], dtype=object)
        noise = np.zeros(pr.n, dtype=object)
        for gi in range(G):
            M = M + np.array(negacyclic_product_z(wc[o, gi], u[0, gi]), dtype=object)
            noise = noise + np.array(negacyclic_product_z(wc[o, gi], e[0, gi]), dtype=object)
        for k in range(pr.n):
            Mk = int(M[k])
            want = (_delta(pr) * (Mk % pr.t) + int(noise[k]) - rq * (Mk // pr.t)) % pr.q
            assert int(phi[0, o, k]) == want, (o, k)


def check_homconv_words(orc):
    """Both words of an output are slot-wise sums of filter x input words
    mod q_l; only b^ carries the mask (HomShare adds a trivial encryption)."""
    pr = TOY
    x_hat, w_hat, r, s, e, res = _conv_case(orc, pr, 2, 10, 3, 16, 50)
    ct, we, me, out = res["ct_in"], res["w_enc"], res["mask_enc"], res["ct_out"]
    Cout, G, K = we.shape[:3]
    for b in range(2):
        for o in range(Cout):
            for l, m in enumerate((pr.q0, pr.q1)):
                for w in range(2):
                    acc = np.zeros(pr.n, dtype=object)
                    for gi in range(G):
                        acc = acc + we[o, gi, 0, l].astype(object) * ct[b, gi, l, w].astype(object)
                    if w == 1:
                        acc = acc + me[b, o, l].astype(object)
                    assert [int(x) % m for x in acc] == [int(x) for x in out[b, o, l, w]]
    # the mask encoding is the scaled trivial encryption: its phase is Delta u_r
    ur = orc.negacyclic(r, pr.t, inverse=True)
    for l, m in enumerate((pr.q0, pr.q1)):
        coeff = orc.negacyclic(me[0, 0, l], m, inverse=True)
        assert [int(x) for x in coeff] == [_delta(pr) * int(v) % m for v in ur[0, 0]]


# ---------------------------------------------------- circuit privacy ---


def check_rerandomize_draws(orc):
    """The server's draws: output ((c0 + i) 3 + w) n + j + 1 of a big-integer
    SplitMix64, mapped by floor(hi32 (2B + 1) / 2^32) - B; every value of the
    ternary rho appears and the flooding e2 spans its range."""
    pr, flood = TOY, 1000
    d = orc.rerand_draws(pr, 3, seed_r=7, flood=flood, ct_index0=4)
    stream = bf.splitmix64_stream(7, (4 + 3) * 3 * pr.n + 1)
    for i in range(3):
        for w, B in enumerate((1, 16, flood)):
            for j in range(pr.n):
                z = stream[((4 + i) * 3 + w) * pr.n + j]
                assert int(d[i, w, j]) == (((z >> 32) * (2 * B + 1)) >> 32) - B
    assert set(np.unique(d[:, 0])) == {-1, 0, 1}
    assert np.abs(d[:, 1]).max() <= 16 and np.abs(d[:, 2]).max() <= flood
    assert d[:, 2].max() > 0.8 * flood and d[:, 2].min() < -0.8 * flood


def check_rerandomize_identity(orc):
    """Re-randomising adds exactly a public-key encryption of zero: with
    pk = Enc(0; e_pk) and draws (rho, e1, e2), the phase grows by
    e_pk rho + e2 - e1 s (mod q) and the a^ word's coefficients by
    a_pk rho + e1 (mod q_l), products in Z[X]/(X^n+1); the message stays."""
    pr, flood = TOY, 5000
    g = _rng(70)
    s = g.integers(-1, 2, size=pr.n).astype(np.int8)
    v = g.integers(0, pr.t, size=(2, pr.n))
    e = np.rint(g.normal(0, 4.0, size=v.shape)).astype(np.int32)
    e_pk = np.rint(g.normal(0, 4.0, size=(1, pr.n))).astype(np.int32)
    pk = orc.encrypt(pr, np.zeros((1, pr.n), np.int64), s, e_pk, seed_a=71)[0]
    ct = orc.encrypt(pr, v, s, e, seed_a=72)
    out = orc.rerandomize(pr, ct, pk, seed_r=73, flood=flood, ct_index0=2)
    d = orc.rerand_draws(pr, 2, seed_r=73, flood=flood, ct_index0=2)
    phi0, phi1 = orc.phase(pr, ct, s), orc.phase(pr, out, s)
    for i in range(2):
        rho, e1, e2 = (d[i, w].astype(np.int64) for w in range(3))
        grow = np.array(negacyclic_product_z(e_pk[0], rho), dtype=object) + e2.astype(object) - np.array(
            negacyclic_product_z(e1, s.astype(np.int64)), dtype=object)
        assert [(int(b) - int(a)) % pr.q for a, b in zip(phi0[i], phi1[i])] == [int(x) % pr.q for x in grow]
        for l, m in enumerate((pr.q0, pr.q1)):
            a_pk = orc.negacyclic(pk[l, 0], m, inverse=True)
            da = orc.negacyclic(((out[i, l, 0].astype(np.int64) - ct[i, l, 0].astype(np.int64)) % m), m, inverse=True)
            want = (negacyclic_product(a_pk, rho % m, m) + e1) % m
            assert np.array_equal(da.astype(np.int64), want)
    assert np.array_equal(orc.decrypt(pr, out, s), v)


def check_rerandomize_table2(orc):
    """Under Table 2's sets, re-randomising a HomConv output with the widest
    flood that leaves room for the product's noise keeps the decryption."""
    for pr in (_sets()[0], _sets()[2]):
        x_hat, w_hat, r, s, e, res = _conv_case(orc, pr, 1, 3, 1, pr.n // 2, 80)
        g = _rng(81)
        pk = orc.encrypt(pr, np.zeros((1, pr.n), np.int64), s,
                         np.rint(g.normal(0, 4.0, size=(1, pr.n))).astype(np.int32), seed_a=82)[0]
        flood = min(_delta(pr) // 16, 2**30)
        out = orc.rerandomize(pr, res["ct_out"], pk, seed_r=83, flood=flood)
        assert np.array_equal(orc.decrypt(pr, out, s), res["v_out"])
        assert not np.array_equal(out[..., 0, :], res["ct_out"][..., 0, :])


# cheapest first (the mutant test stops at the first failing pin)
ALL_CHECKS = [
    check_params_against_table2,
    check_psi,
    check_negacyclic_definition,
    check_pack_and_fold,
    check_decryption_rounding,
    check_public_constants,
    check_homconv_noise_identity,
    check_homconv_words,
    check_rerandomize_draws,
    check_rerandomize_identity,
    check_secure_conv_plaintext,
    check_rerandomize_table2,
    check_roundtrip,
    check_convolution_theorem,
    check_enc_phase_exact,
]
