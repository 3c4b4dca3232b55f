"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Each ``check_*`` takes an oracle object (``oracle.Oracle``) and raises
AssertionError when the oracle disagrees with something other than itself:
brute force with Python integers, closed forms, invariants, numpy library
routines (float64 FFT, uint64 matmul), the paper's printed moduli, and a
published generator's known answers. ``tests/test_oracle_pins.py`` runs them
on the committed oracle; ``tests/test_oracle_mutants.py`` plants plausible
mistakes in copies of the oracle source and shows each one is caught.
"""
from __future__ import annotations

import os

import numpy as np

import oracle
from tests import bruteforce as bf
from paper_2003_05328_amd import synth

P = 65537
M64 = 1 << 64
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- field ---


def check_roots(orc):
    # 3 is a primitive root of every Fermat prime 2^(2^k)+1 > 3 (Pepin's theorem)
    assert orc.primitive_root(P) == 3
    assert orc.primitive_root(257) == 3
    for p in (P, 12289, 257, 97, 193):
        N = 2
        while (p - 1) % N == 0 and N <= 4096:
            w = orc.root_of_unity(p, N)
            wi = orc.root_of_unity(p, N, True)
            assert pow(w, N, p) == 1, (p, N)
            assert pow(w, N // 2, p) == p - 1, (p, N)  # order exactly N
            assert w * wi % p == 1
            N *= 2
    # brute-force generator search agrees on small primes
    for p in (17, 97, 193, 257):
        for N in (2, 4, 8, 16):
            if (p - 1) % N == 0:
                assert orc.root_of_unity(p, N) == bf.brute_root(p, N)
                assert orc.root_of_unity(p, N, True) == bf.brute_root(p, N, True)


def check_delta(orc):
    # 2^64 - 1 = (2^16 + 1)(2^48 - 2^32 + 2^16 - 1): Delta * p = 2^64 - 1 for p = 65537
    assert orc.delta(P) == 0xFFFF0000FFFF == 2**48 - 2**32 + 2**16 - 1
    assert orc.delta(P) * P == M64 - 1
    for p in (12289, 147457, 2363393, 257):
        d = orc.delta(p)
        assert d * p <= M64 < (d + 1) * p


def check_table2(orc):
    """The paper's Table 2 moduli meet the constraints of Sec. 5.2 / 6.4."""
    rows = []
    with open(os.path.join(GOLDEN, "table2_moduli.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, pn, pe, lgq, n = line.split()
                rows.append((name, int(pn), int(pe), int(n)))
    assert len(rows) == 3
    for name, pn, pe, n in rows:
        assert orc.is_prime(pe), name
        assert pe % n == 1, name
        assert pe >= pn, name
        assert pn % 3 == 1, name
        # p_E is the smallest prime >= p_N with p_E = 1 mod n
        c = pn + ((1 - pn) % n)
        while not orc.is_prime(c):
            c += n
        assert c == pe, (name, c, pe)
    assert rows[2][1] >= 2**12 * 2**6 * 9
    assert not orc.is_prime(65535) and orc.is_prime(P) and not orc.is_prime(1)  # 65535 = 3*5*17*257


# ------------------------------------------------------------ transforms ---


def check_dft_bruteforce(orc):
    g = _rng(1)
    for p in (257, P):
        for H, W in ((2, 2), (2, 4), (4, 2), (4, 4), (4, 8), (8, 8)):
            x = g.integers(0, p, size=(H, W)).astype(np.uint32)
            for inv in (False, True):
                ref = np.array(bf.brute_dft2d(x.tolist(), p, inv), dtype=np.uint32)
                assert np.array_equal(orc.dft2d_direct(x, p, inv), ref), (p, H, W, inv)
                assert np.array_equal(orc.ntt2d(x, p, inv), ref), (p, H, W, inv)


def check_basis_vectors(orc):
    p = P
    for H, W in ((4, 4), (4, 8), (8, 4), (16, 16)):
        wH, wW = bf.brute_root(p, H), bf.brute_root(p, W)
        basis = np.zeros((H * W, H, W), dtype=np.uint32)
        for a in range(H):
            for b in range(W):
                basis[a * W + b, a, b] = 1
        out = orc.ntt2d(basis, p)
        k1 = np.arange(H)[:, None]
        k2 = np.arange(W)[None, :]
        for a in range(H):
            for b in range(W):
                exp = np.array([[pow(wH, a * i, p) * pow(wW, b * j, p) % p for j in range(W)] for i in range(H)])
                assert np.array_equal(out[a * W + b], exp), (H, W, a, b)
        del k1, k2
        # delta at the origin transforms to all ones; a constant c to (c F, 0, ..., 0)
        assert np.all(out[0] == 1)
        c = np.full((H, W), 1234, dtype=np.uint32)
        X = orc.ntt2d(c, p)
        assert X[0, 0] == 1234 * H * W % p and np.count_nonzero(X) == 1


def check_roundtrip(orc):
    g = _rng(2)
    sizes = [2, 4, 8, 16, 32, 64, 128]
    for H in sizes:
        for W in sizes:
            if H * W > 8192 and (H, W) != (128, 128):
                continue
            x = g.integers(0, P, size=(2, H, W)).astype(np.uint32)
            X = orc.ntt2d(x, P)
            assert np.array_equal(orc.ntt2d(X, P, inverse=True), x), (H, W)


def check_linearity(orc):
    g = _rng(3)
    x = g.integers(0, P, size=(8, 16)).astype(np.uint32)
    y = g.integers(0, P, size=(8, 16)).astype(np.uint32)
    a = 777
    lhs = orc.ntt2d(((a * x.astype(np.int64) + y) % P).astype(np.uint32), P)
    rhs = (a * orc.ntt2d(x, P).astype(np.int64) + orc.ntt2d(y, P)) % P
    assert np.array_equal(lhs, rhs)


def _fft_conv(x, w, H, W, p):
    """numpy float64 FFT circular convolution summed over channels, rounded, mod p."""
    B, Cin = x.shape[:2]
    Cout, _, kh, kw = w.shape
    wp = np.zeros((Cout, Cin, H, W))
    wp[:, :, :kh, :kw] = w
    X = np.fft.fft2(x.astype(np.float64))
    Wf = np.fft.fft2(wp)
    y = np.real(np.fft.ifft2(np.einsum("bihw,oihw->bohw", X, Wf)))
    return (np.rint(y).astype(np.int64) % p).astype(np.uint32)


def check_conv_theorem(orc):
    g = _rng(4)
    for p, (H, W), (Cin, Cout), (kh, kw) in (
        (P, (16, 16), (3, 2), (3, 3)),
        (P, (8, 16), (2, 3), (3, 2)),
        (12289, (16, 16), (2, 2), (5, 5)),
        (P, (32, 32), (4, 3), (7, 7)),
    ):
        x = g.integers(0, p, size=(1, Cin, H, W)).astype(np.uint32)
        w = g.integers(-8, 9, size=(Cout, Cin, kh, kw)).astype(np.int32)
        direct = orc.cyclic_conv(x, w, p)
        assert np.array_equal(direct, _fft_conv(x, w, H, W, p)), (p, H, W)
        xh = orc.ntt2d(x, p).reshape(1, 1, Cin, H * W).astype(object)
        wh = orc.weight_prep(w, H, W, p).astype(object)
        prod = (xh * wh[None]).sum(axis=2) % p  # [1][Cout][F]
        y = orc.ntt2d(prod.astype(np.uint32).reshape(1, Cout, H, W), p, inverse=True)
        assert np.array_equal(y, direct), (p, H, W)
    # single channel against Python brute force
    x = g.integers(0, 256, size=(4, 4))
    w = g.integers(-8, 9, size=(2, 3))
    ref = np.array(bf.brute_cyclic_conv(x.tolist(), w.tolist(), P))
    got = orc.cyclic_conv(x[None, None].astype(np.uint32), w[None, None].astype(np.int32), P)[0, 0]
    assert np.array_equal(got, ref)


def check_weight_prep(orc):
    g = _rng(5)
    w = g.integers(-8, 9, size=(3, 2, 3, 2)).astype(np.int32)
    H, W = 8, 16
    pad = np.zeros((3, 2, H, W), dtype=np.int64)
    pad[:, :, :3, :2] = w
    ref = np.array(
        [[bf.brute_dft2d((pad[o, i] % P).tolist(), P) for i in range(2)] for o in range(3)], dtype=np.uint32
    ).reshape(3, 2, H * W)
    assert np.array_equal(orc.weight_prep(w, H, W, P), ref)


# ------------------------------------------------------------------ LWE ---


def check_splitmix(orc):
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as fh:
        kat = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for k, hx in kat:
        assert orc.splitmix64(0, int(k)) == int(hx, 16)
    for seed in (0, 1, 0xDEADBEEF12345678, 2**64 - 1):
        stream = bf.splitmix64_stream(seed, 300)
        for k in (1, 2, 3, 57, 300):
            assert orc.splitmix64(seed, k) == stream[k - 1], (seed, k)


def check_encrypt(orc):
    g = _rng(6)
    N, n, seed_a, c0 = 20, 16, 0x0123456789ABCDEF, 5
    m = g.integers(0, P, size=N).astype(np.uint32)
    s = synth.ternary(7, n)
    e = synth.rounded_gaussian(8, N)
    ct = orc.encrypt(m, s, e, seed_a, P, ct_index0=c0)
    stream = bf.splitmix64_stream(seed_a, (c0 + N) * n)
    D = bf.brute_delta(P)
    for c in range(N):
        a = [int(v) for v in ct[c, :n]]
        assert a == stream[(c0 + c) * n : (c0 + c + 1) * n]
        dot = sum(int(s[j]) * a[j] for j in range(n))
        assert (int(ct[c, n]) - dot - D * int(m[c]) - int(e[c])) % M64 == 0
    # encrypting a slice with its global index gives the same words
    part = orc.encrypt(m[7:], s, e[7:], seed_a, P, ct_index0=c0 + 7)
    assert np.array_equal(part, ct[7:])
    # word-major storage of B x C x F plaintexts: ciphertext (b, c, f) is number
    # q = (b F + f) C + c, its word j sits at ct[b][f][j][c]
    B, C, F = 2, 3, 5
    m3 = g.integers(0, P, size=(B, C, F)).astype(np.uint32)
    e3 = synth.rounded_gaussian(9, (B, C, F))
    ct3 = orc.encrypt(m3, s, e3, seed_a, P)
    assert ct3.shape == (B, F, n + 1, C)
    stream = bf.splitmix64_stream(seed_a, B * C * F * n)
    for b in range(B):
        for c in range(C):
            for f in range(F):
                q = (b * F + f) * C + c
                a = [int(v) for v in ct3[b, f, :n, c]]
                assert a == stream[q * n : (q + 1) * n]
                dot = sum(int(s[j]) * a[j] for j in range(n))
                assert (int(ct3[b, f, n, c]) - dot - D * int(m3[b, c, f]) - int(e3[b, c, f])) % M64 == 0
    assert np.array_equal(orc.decrypt(ct3, s, P), m3)


def check_decrypt_exhaustive(orc):
    """Dec(Enc(m)) == m for every m in Z_p, with errors up to 12.5 sigma."""
    n = 16
    m = np.arange(P, dtype=np.uint32)
    s = synth.ternary(9, n)
    e = np.clip(synth.rounded_gaussian(10, P) * 4, -40, 40).astype(np.int32)
    e[0], e[1], e[-1] = -40, 40, 40  # m = 0 with negative noise wraps below 0
    ct = orc.encrypt(m, s, e, 99, P)
    assert np.array_equal(orc.decrypt(ct, s, P), m)


def check_decode_rounding(orc):
    """Dec's rounding against exact rationals, at the decision boundaries."""
    D = bf.brute_delta(P)
    n = 4
    s = np.zeros(n, dtype=np.int8)  # phase = b
    phis = []
    for m in (0, 1, 2, 32768, 65535, 65536):
        e_hi = (2**63 - 1 + m) // P  # largest error still decoding to m
        e_lo = -((2**63 - m) // P)  # smallest error still decoding to m
        for E in (e_hi, e_hi + 1, e_lo, e_lo - 1, 0, 40, -40):
            phis.append((D * m + E) % M64)
    g = _rng(11)
    phis += [int(v) for v in g.integers(0, 2**64, size=2000, dtype=np.uint64)]
    phis += [0, 1, 2**63 - 1, 2**63, 2**64 - 1]
    ct = np.zeros((len(phis), n + 1), dtype=np.uint64)
    ct[:, n] = np.array(phis, dtype=np.uint64)
    got = orc.decrypt(ct, s, P)
    exp = np.array([bf.brute_decode(v, P) for v in phis], dtype=np.uint32)
    assert np.array_equal(got, exp)


# -------------------------------------------------------------- HomConv ---


def check_homconv_numpy(orc):
    g = _rng(12)
    B, Cin, Cout, F, n = 2, 5, 3, 8, 7
    ct = g.integers(0, 2**64, size=(B, F, n + 1, Cin), dtype=np.uint64)
    w = g.integers(0, P, size=(Cout, Cin, F)).astype(np.uint32)
    w[0, 0, 0] = P - 1
    r = g.integers(0, P, size=(B, Cout, F)).astype(np.uint32)
    out = orc.homconv(ct, w, r, P)
    assert out.shape == (B, F, n + 1, Cout)
    D = np.uint64(bf.brute_delta(P))
    for b in range(B):
        for f in range(F):
            ref = ct[b, f] @ w[:, :, f].T.astype(np.uint64)  # [n+1][Cout], uint64 matmul wraps mod 2^64
            ref[n, :] += D * r[b, :, f].astype(np.uint64)
            assert np.array_equal(out[b, f], ref), (b, f)
    sel = np.array([[1, 2, 7], [0, 0, 0], [1, 0, 3]])
    rows = orc.homconv_select(ct, w, r, sel, P)
    for k, (b, o, f) in enumerate(sel):
        assert np.array_equal(rows[k], out[b, f, :, o])


def check_homconv_special(orc):
    g = _rng(13)
    ct = g.integers(0, 2**64, size=(1, 4, 9, 1), dtype=np.uint64)
    one = np.ones((1, 1, 4), dtype=np.uint32)
    zero_r = np.zeros((1, 1, 4), dtype=np.uint32)
    assert np.array_equal(orc.homconv(ct, one, zero_r, P), ct)
    r = g.integers(0, P, size=(1, 2, 4)).astype(np.uint32)
    out = orc.homconv(ct, np.zeros((2, 1, 4), dtype=np.uint32), r, P)
    assert np.all(out[:, :, :8, :] == 0)
    assert np.array_equal(out[0, :, 8, :], (np.uint64(bf.brute_delta(P)) * r[0].T.astype(np.uint64)))


def _small_layer(seed, H=8, W=8, Cin=3, Cout=2, k=3, n=32, B=1, hidden=False):
    S = synth.LayerShape(H=H, W=W, Cin=Cin, Cout=Cout, kh=k, kw=k, n=n, B=B, hidden=hidden)
    return synth.generate(S, P, seed)


def check_noise_identity(orc):
    """phi_out - Delta*m_out equals sum_i W^ e_i - floor(M/p) exactly, with
    M = sum_i W^ x^_i + r the integer plaintext before reduction."""
    inp = _small_layer(14, Cin=4, Cout=3, n=24, B=2)
    S = inp.shape
    out = orc.fdsc_round0(inp, P)
    D = bf.brute_delta(P)
    xh = out["x_hat"].astype(object)
    wh = out["w_hat"].astype(object)
    e = inp.e.astype(object)
    for b in range(S.B):
        for o in range(S.Cout):
            for f in range(S.F):
                Mi = sum(wh[o, i, f] * xh[b, i, f] for i in range(S.Cin)) + int(inp.r[b, o, f])
                mo = Mi % P
                E = sum(wh[o, i, f] * e[b, i, f] for i in range(S.Cin)) - Mi // P
                phi = orc.phase(out["ct_out"][b, f, :, o], inp.s)
                assert (phi - D * mo - E) % M64 == 0
                assert int(out["m"][b, o, f]) == mo
                assert abs(E * P - mo) < 2**63


def check_end_to_end(orc):
    """INTT2D(Dec(HomConv(Enc(NTT2D(x))))) + INTT2D(-r) = x * w mod p
    (the correctness statement of Sec. 4.1.1 / Appendix A, p_A = p_N)."""
    for seed, kw in ((15, {}), (16, dict(H=16, W=16, Cin=3, Cout=8, n=64)), (17, dict(H=8, W=16, k=5, hidden=True))):
        inp = _small_layer(seed, **kw)
        out = orc.fdsc_round0(inp, P)
        y = (out["s_a"].astype(np.int64) + out["s_b"]) % P
        conv = orc.cyclic_conv(inp.x, inp.w, P)
        assert np.array_equal(y, conv), seed
        assert np.array_equal(conv, _fft_conv(inp.x, inp.w, inp.shape.H, inp.shape.W, P))


def check_homrec(orc):
    """HomRec (Eq. homrec; Fig. 2's re-entry of the server's share): Dec(HomRec(Enc(m), s)) = m + s
    mod p at edge residues and inside; since Delta p = 2^64 - 1 the phase is
    Delta ((m + s) mod p) plus the encryption error, minus 1 exactly when
    m + s wraps past p; the a-words are untouched. Ciphertexts of several
    channels and frequencies check that each share lands on its own b word."""
    vals = np.array([0, 1, 2, 32767, 32768, 32769, P - 2, P - 1], dtype=np.int64)
    m = np.repeat(vals, vals.size)
    s = np.tile(vals, vals.size)
    n, Cc, F = 16, 4, 16  # 64 ciphertexts as [1][F][n+1][C]
    g = _rng(18)
    key = g.integers(-1, 2, size=n).astype(np.int8)
    e = g.integers(-40, 41, size=(1, Cc, F)).astype(np.int32)
    mm = m.reshape(1, Cc, F).astype(np.uint32)
    ct = orc.encrypt(mm, key, e, 91, P)
    rec = orc.homrec(ct, s.reshape(1, Cc, F).astype(np.uint32), P)
    assert np.array_equal(rec[:, :, :n, :], ct[:, :, :n, :])
    ss = s.reshape(1, Cc, F)
    assert np.array_equal(orc.decrypt(rec, key, P).astype(np.int64), (mm.astype(np.int64) + ss) % P)
    D = bf.brute_delta(P)
    for c in range(Cc):
        for f in range(F):
            tot = int(mm[0, c, f]) + int(ss[0, c, f])
            phase = orc.phase(rec[0, f, :, c], key)
            assert phase == (D * (tot % P) + int(e[0, c, f]) - int(tot >= P)) % M64


def check_reshare(orc):
    """The stand-in for the oblivious activation between the rounds of Fig. 2 (in the
    clear): the shares after it add up to f(s_A + s_B) mod p, f the identity
    or the square, edge residues included."""
    g = _rng(19)
    s_a = g.integers(0, P, size=300).astype(np.uint32)
    s_b = g.integers(0, P, size=300).astype(np.uint32)
    s_b2 = g.integers(0, P, size=300).astype(np.uint32)
    s_a[:3], s_b[:3], s_b2[:3] = P - 1, P - 1, [0, P - 1, 1]
    for act in (0, 1):
        out = orc.reshare(s_a, s_b, s_b2, act, P)
        assert int(out.max()) < P
        for k in range(300):
            y = (int(s_a[k]) + int(s_b[k])) % P
            assert (int(out[k]) + int(s_b2[k])) % P == (y if act == 0 else y * y % P)


def check_chained_rounds(orc):
    """Round 0, the activation stand-in, Enc of the client's new share,
    HomRec with the server's transformed share, and round 1: the final shares
    add up to conv(f(conv(x, w0)), w1) mod p (two rounds of Fig. 2; Eq.
    dft_convolution)."""
    S0 = synth.LayerShape(H=8, W=4, Cin=2, Cout=3, kh=3, kw=2, n=24, B=2)
    S1 = synth.LayerShape(H=8, W=4, Cin=3, Cout=2, kh=2, kw=3, n=24, B=2, hidden=True)
    inp0, inp1 = synth.generate(S0, P, 31), synth.generate(S1, P, 32)
    r0 = orc.fdsc_round0(inp0, P)
    s_b1 = synth.uniform_u32(33, (S1.B, S1.Cin, S1.H, S1.W), P)
    conv0 = orc.cyclic_conv(inp0.x, inp0.w, P).astype(np.int64)
    for act in (0, 1):
        r1 = orc.fdsc_round1(r0, inp1, s_b1, act, P)
        u1 = conv0 if act == 0 else conv0 * conv0 % P
        want = _fft_conv(u1.astype(np.uint32), inp1.w, S1.H, S1.W, P)
        got = (r1["s_a"].astype(np.int64) + r1["s_b"]) % P
        assert np.array_equal(got.reshape(want.shape), want), act


def check_seeded(orc):
    """Seeded ciphertexts (Sec. 5.1: the ciphertexts' public constants are
    generated offline, so only the b words travel). The expansion's a-words
    are the generator's stream at the stated counters (a stateful big-int
    generator, independent of the oracle's); its b row is the given words; Enc
    followed by dropping the a-words and expanding again is the identity; and
    HomConv of the expansion decrypts to sum_i W^ m + r."""
    g = _rng(23)
    B, C, F, n, seed_a, c0 = 2, 3, 5, 16, 0x0F1E2D3C4B5A6978, 11
    bw = synth.uniform_u64(24, (B, F, C))
    ct = orc.expand_seeded(bw, n, seed_a, ct_index0=c0)
    assert ct.shape == (B, F, n + 1, C)
    stream = bf.splitmix64_stream(seed_a, (c0 + B * C * F) * n)
    for b in range(B):
        for c in range(C):
            for f in range(F):
                q = (b * F + f) * C + c
                assert [int(v) for v in ct[b, f, :n, c]] == stream[(c0 + q) * n : (c0 + q + 1) * n]
                assert int(ct[b, f, n, c]) == int(bw[b, f, c])
    m = g.integers(0, P, size=(B, C, F)).astype(np.uint32)
    s = synth.ternary(25, n)
    e = synth.rounded_gaussian(26, (B, C, F))
    full = orc.encrypt(m, s, e, seed_a, P, ct_index0=c0)
    b_only = orc.encrypt_seeded(m, s, e, seed_a, P, ct_index0=c0)
    assert b_only.shape == (B, F, C)
    assert np.array_equal(orc.expand_seeded(b_only, n, seed_a, ct_index0=c0), full)
    Cout = 4
    w_hat = g.integers(0, P, size=(Cout, C, F)).astype(np.uint32)
    r = g.integers(0, P, size=(B, Cout, F)).astype(np.uint32)
    out = orc.homconv_seeded(b_only, n, seed_a, w_hat, r, P, ct_index0=c0)
    want = (np.einsum("oif,bif->bof", w_hat.astype(np.int64), m.astype(np.int64)) + r) % P
    assert np.array_equal(orc.decrypt(out, s, P).astype(np.int64), want)


def check_cdt_exact(orc):
    """The sampler's thresholds exactly: T[k] = floor(2^48 erf((k + 1/2) /
    (sigma sqrt 2))) for every k < 32, with erf from mpmath at 60 digits (an
    implementation independent of the oracle's decimal series). Every
    2^48 erf value checked lies at least 1e-30 from an integer, so the floor
    taken at this precision is certain."""
    import mpmath

    T = oracle.cdt_table()
    assert len(T) == oracle.CDT_SIZE
    with mpmath.workdps(60):
        sigma = mpmath.mpf(oracle.SIGMA_NUM) / oracle.SIGMA_DEN
        for k, t in enumerate(T):
            v = mpmath.ldexp(mpmath.erf((k + mpmath.mpf(1) / 2) / (sigma * mpmath.sqrt(2))), oracle.CDT_BITS)
            fl = int(mpmath.floor(v))
            assert mpmath.mpf(10) ** -30 < v - fl < 1 - mpmath.mpf(10) ** -30, k
            assert t == fl, (k, t, fl)


def check_noise_sampler(orc):
    """The rounded-Gaussian error sampler (sigma 3.2): its thresholds against
    the library erf, its draws against a stateful big-int generator and a
    plain lookup, and the moments and zero mass of 200,000 draws against the
    rounded Gaussian's (variance sigma^2 + 1/12 to first order)."""
    import math

    T = oracle.cdt_table()
    sigma = oracle.SIGMA_NUM / oracle.SIGMA_DEN
    assert len(T) == oracle.CDT_SIZE and T[-1] == 2**oracle.CDT_BITS - 1
    for k, t in enumerate(T):
        assert abs(t / 2**oracle.CDT_BITS - math.erf((k + 0.5) / (sigma * math.sqrt(2)))) < 1e-14, k
        if k:
            assert t >= T[k - 1]
    # indexing: error (b, c, f) from generator output ct_index0 + (b F + f) C + c + 1
    B, C, F, seed_e, c0 = 2, 3, 5, 0xC0FFEE1234, 9
    e = orc.sample_errors(seed_e, B, C, F, ct_index0=c0)
    stream = bf.splitmix64_stream(seed_e, c0 + B * C * F)
    for b in range(B):
        for c in range(C):
            for f in range(F):
                u = stream[c0 + (b * F + f) * C + c]
                v = (u >> 15) % 2**48
                mag = sum(1 for t in T if t <= v)
                assert int(e[b, c, f]) == (-mag if u >> 63 and mag else mag), (b, c, f)
    # distribution
    N = 200_000
    x = orc.sample_errors(77, 1, 1, N).astype(np.float64).ravel()
    var = sigma**2 + 1 / 12
    assert abs(x.mean()) < 4 * math.sqrt(var / N)
    assert abs(x.var() / var - 1) < 0.02
    p0 = math.erf(0.5 / (sigma * math.sqrt(2)))
    assert abs((x == 0).mean() - p0) < 4 * math.sqrt(p0 * (1 - p0) / N)
    assert abs((x > 0).mean() - (x < 0).mean()) < 0.01
    assert np.abs(x).max() <= 8 * sigma


ALL_CHECKS = [
    check_roots,
    check_delta,
    check_table2,
    check_dft_bruteforce,
    check_basis_vectors,
    check_roundtrip,
    check_linearity,
    check_conv_theorem,
    check_weight_prep,
    check_splitmix,
    check_encrypt,
    check_decrypt_exhaustive,
    check_decode_rounding,
    check_homconv_numpy,
    check_homconv_special,
    check_noise_identity,
    check_end_to_end,
    check_homrec,
    check_reshare,
    check_chained_rounds,
    check_seeded,
    check_cdt_exact,
    check_noise_sampler,
]
