"""GPU parity: every HIP entry point against the CPU oracle, bit for bit.

Small cases span several workgroup tiles and ragged tails and are compared
element by element; full-size layers are compared on outputs the oracle
computes one by one (sampled ciphertext rows) and on properties that hold at
any size (exact decryption, s_A + s_B = x (*) w mod p).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05328_amd import configs, synth
from paper_2003_05328_amd.ensei import Context, EnseiError
from tests.gpu_helpers import P, ct_words, dev, host, oracle_ct_in_rows, oracle_ct_out_row

pytestmark = pytest.mark.gpu

SIZES = [2, 4, 8, 16, 32, 64, 128]


@pytest.fixture(scope="module")
def ctx():
    c = Context(P, 0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    o = oracle.default()
    o.set_threads(16)
    return o


def _batch_for(H, W):
    T = max(1, 256 // max(H, W)) if max(H, W) < 128 else 1
    return 2 * T + 3  # two full workgroups and a ragged one


# ------------------------------------------------------------- transforms ---


@pytest.mark.parametrize("H", SIZES)
@pytest.mark.parametrize("W", SIZES)
def test_ntt2d_intt2d(ctx, orc, H, W):
    batch = _batch_for(H, W) if H * W <= 4096 else 3
    x = synth.uniform_u32(1000 + H * 131 + W, (batch, H, W), P)
    x[0] = P - 1  # largest residue everywhere
    X = host(ctx.ntt2d(dev(x)))
    assert np.array_equal(X.reshape(batch, H, W), orc.ntt2d(x, P))
    Y = synth.uniform_u32(2000 + H * 131 + W, (batch, H * W), P)
    y = host(ctx.intt2d(dev(Y), H, W))
    assert np.array_equal(y, orc.ntt2d(Y.reshape(batch, H, W), P, inverse=True))


@pytest.mark.parametrize("H,W", [(8, 8), (16, 16), (32, 32), (64, 64), (8, 64), (64, 16)])
def test_ntt2d_group_boundaries(ctx, orc, H, W):
    """A workgroup transforms T grids: batches that end inside a workgroup's
    group, on a whole number of groups, and a single grid."""
    T = max(1, 256 // max(H, W))
    for batch in (3 * T + 1, 4 * T, 1):
        x = synth.uniform_u32(3000 + H * 7 + W + batch, (batch, H, W), P)
        assert np.array_equal(host(ctx.ntt2d(dev(x))).reshape(batch, H, W), orc.ntt2d(x, P)), batch
        Y = synth.uniform_u32(4000 + H * 7 + W + batch, (batch, H * W), P)
        y = host(ctx.intt2d(dev(Y), H, W))
        assert np.array_equal(y, orc.ntt2d(Y.reshape(batch, H, W), P, inverse=True)), batch


def test_ntt2d_in_place_and_roundtrip(ctx, orc):
    # 37 grids of 32 x 32: groups of 4 channels per workgroup, the last ragged
    x = synth.uniform_u32(7, (37, 32, 32), P)
    t = dev(x)
    ctx.ntt2d(t, out=t.view(37, 1024))
    assert np.array_equal(host(t), orc.ntt2d(x, P))
    back = ctx.intt2d(t.view(37, 1024), 32, 32)
    assert np.array_equal(host(back), x)


def test_server_share(ctx, orc):
    r = synth.uniform_u32(8, (5, 3, 256), P)
    got = host(ctx.server_share(dev(r), 16, 16))
    assert np.array_equal(got, orc.server_share(r, 16, 16, P))


@pytest.mark.parametrize("Cout,Cin,kh,kw,H,W", [(8, 3, 3, 3, 16, 16), (5, 7, 7, 7, 32, 32), (3, 2, 3, 5, 8, 16),
                                                (2, 2, 1, 1, 128, 128), (4, 3, 4, 4, 4, 4)])
def test_weight_prep(ctx, orc, Cout, Cin, kh, kw, H, W):
    g = np.random.default_rng(Cout * 100 + Cin)
    w = g.integers(-200000, 200000, size=(Cout, Cin, kh, kw)).astype(np.int32)
    w.flat[0] = -(2**31)
    w.flat[-1] = 2**31 - 1
    got = host(ctx.weight_prep(dev(w), H, W))
    assert np.array_equal(got, orc.weight_prep(w, H, W, P))


# -------------------------------------------------------------------- LWE ---


@pytest.mark.parametrize("n,num_ct,c0", [(1, 5, 0), (16, 77, 3), (63, 130, 0), (64, 64, 2**40), (65, 257, 11),
                                         (512, 300, 0), (1024, 1000, 123456), (16384, 70, 7)])
def test_encrypt_decrypt(ctx, orc, n, num_ct, c0):
    m = synth.uniform_u32(n, num_ct, P)
    m[:2] = [0, P - 1]
    s = synth.ternary(n + 1, n)
    e = synth.rounded_gaussian(n + 2, num_ct)
    seed_a = 0xC0FFEE ^ n
    ct = ctx.encrypt(dev(m), dev(s), dev(e), seed_a, ct_index0=c0)
    ref = orc.encrypt(m, s, e, seed_a, P, ct_index0=c0)
    assert np.array_equal(host(ct), ref)
    assert np.array_equal(host(ctx.decrypt(ct, dev(s))), m)
    # decryption of arbitrary words (not only fresh encryptions)
    junk = synth.uniform_u64(n + 3, (num_ct, n + 1))
    assert np.array_equal(host(ctx.decrypt(dev(junk), dev(s))), orc.decrypt(junk, s, P))


@pytest.mark.parametrize("B,C,F,n", [(2, 3, 50, 64), (1, 64, 17, 100), (2, 70, 5, 33), (1, 130, 3, 1024),
                                     (1, 1, 700, 16), (3, 21, 7, 1)])
def test_encrypt_decrypt_word_major(ctx, orc, B, C, F, n):
    """Channel groups of one frequency, several frequencies per group (C < 64),
    partial channel blocks (C > 64) and ragged word ranges."""
    m = synth.uniform_u32(B * C, (B, C, F), P)
    s = synth.ternary(C + 1, n)
    e = synth.rounded_gaussian(C + 2, (B, C, F))
    ct = ctx.encrypt(dev(m), dev(s), dev(e), 77, ct_index0=5)
    ref = orc.encrypt(m, s, e, 77, P, ct_index0=5)
    assert np.array_equal(host(ct), ref)
    assert np.array_equal(host(ctx.decrypt(ct, dev(s))), m)
    junk = synth.uniform_u64(C + 3, (B, F, n + 1, C))
    assert np.array_equal(host(ctx.decrypt(dev(junk), dev(s))), orc.decrypt(junk, s, P))


# ---------------------------------------------------------------- HomConv ---

HOMCONV_CASES = [
    # B, Cin, Cout, F, n
    (1, 1, 1, 1, 1),
    (1, 3, 8, 16, 63),
    (2, 3, 8, 5, 64),
    (1, 16, 16, 3, 65),
    (1, 17, 17, 4, 127),
    (2, 33, 40, 2, 128),
    (1, 64, 64, 3, 129),
    (1, 65, 33, 2, 200),
    (1, 130, 70, 2, 64),
    (1, 256, 512, 1, 30),
    # more tiles than resident workgroups: every block walks many (tile, K step) units
    (1, 70, 64, 300, 130),
    (2, 130, 20, 150, 64),
]


def _homconv_inputs(B, Cin, Cout, F, n, seed):
    ct = synth.uniform_u64(seed, (B, F, n + 1, Cin))
    w = synth.uniform_u32(seed + 1, (Cout, Cin, F), P)
    w.flat[0] = P - 1
    w.flat[-1] = 0
    if w.size > 2:
        w.flat[1] = 65536 % P if P > 65536 else P - 2
    r = synth.uniform_u32(seed + 2, (B, Cout, F), P)
    return ct, w, r


@pytest.mark.parametrize("B,Cin,Cout,F,n", HOMCONV_CASES)
def test_homconv_mfma(ctx, orc, B, Cin, Cout, F, n):
    ct, w, r = _homconv_inputs(B, Cin, Cout, F, n, 31 * Cin + Cout)
    ref = orc.homconv(ct, w, r, P)
    pack = ctx.pack_weights(dev(w))
    got = host(ctx.homconv(dev(ct), pack, dev(r), Cout))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("B,Cin,Cout,F,n", HOMCONV_CASES)
def test_homconv_valu(ctx, orc, B, Cin, Cout, F, n):
    ct, w, r = _homconv_inputs(B, Cin, Cout, F, n, 37 * Cin + Cout)
    got = host(ctx.homconv_valu(dev(ct), dev(w), dev(r)))
    assert np.array_equal(got, orc.homconv(ct, w, r, P))


# One K step and one row tile (48 <= Cin <= 64, Cout <= 64), the shape of the
# 64 -> 64 layers: channel groups straddling Cin, odd Cout, one output row,
# the b word first, last or alone in its column tile, and workgroup ranges
# that cross frequencies and images.
SINGLE_STEP_CASES = [
    # B, Cin, Cout, F, n
    (1, 48, 64, 5, 100),
    (2, 64, 64, 7, 31),
    (1, 57, 33, 4, 64),
    (1, 64, 1, 2, 16),
    (3, 50, 17, 300, 40),
    (1, 64, 64, 1024, 255),
]


@pytest.mark.parametrize("B,Cin,Cout,F,n", SINGLE_STEP_CASES)
def test_homconv_single_step(ctx, orc, B, Cin, Cout, F, n):
    ct, w, r = _homconv_inputs(B, Cin, Cout, F, n, 47 * Cin + Cout + n)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


def test_homconv_single_step_extreme_digits(ctx, orc):
    """Digits -128 and +127 against limbs -128, -127, 1 and p - 1 with one K step of 64 channels."""
    B, Cin, Cout, F, n = 2, 64, 64, 3, 40
    ct = np.full((B, F, n + 1, Cin), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    ct[:, :, 1::2, :32] = 0x7F7F7F7F7F7F7F7F
    ct[:, :, ::5, :] = 2**64 - 1
    w = np.full((Cout, Cin, F), 0x8080, dtype=np.uint32)
    w[1::3] = P - 1
    r = np.full((B, Cout, F), P - 1, dtype=np.uint32)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


# Layers with several 64-row output tiles, at most 256 input channels and at
# least four (row tile, K step) pairs take the deep kernel (a block's digit
# planes of every K step held in LDS, all row tiles contracted from them): one
# to four K steps, ragged channel groups and columns, odd Cout, more blocks
# than workgroups; Cin = 257 falls back to the streaming kernel.
DEEP_CASES = [
    # B, Cin, Cout, F, n
    (1, 48, 300, 3, 70),
    (2, 100, 128, 256, 64),
    (1, 100, 129, 4, 90),
    (2, 256, 130, 5, 129),
    (1, 200, 256, 17, 63),
    (1, 130, 512, 2, 40),
    (1, 257, 70, 2, 40),
]


@pytest.mark.parametrize("B,Cin,Cout,F,n", DEEP_CASES)
def test_homconv_deep(ctx, orc, B, Cin, Cout, F, n):
    ct, w, r = _homconv_inputs(B, Cin, Cout, F, n, 43 * Cin + Cout + n)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("Cin", [169, 170])
def test_homconv_deep_extreme_digits(ctx, orc, Cin):
    """Largest same-sign shift sums on the deep kernel, both sides of the
    32-bit partial recombination bound."""
    B, Cout, F, n = 1, 130, 2, 70
    ct = np.full((B, F, n + 1, Cin), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    ct[:, :, 1::2, : Cin // 2] = 0x7F7F7F7F7F7F7F7F
    w = np.full((Cout, Cin, F), 0x8080, dtype=np.uint32)
    w[1::2] = P - 1
    r = np.full((B, Cout, F), 12345, dtype=np.uint32)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


# Inputs of at most 16 channels take the narrow kernel (one wave per unit of
# 16 words, no LDS): channel counts of each of its widths, odd Cout (8-byte
# stores), several row tiles, the b word first, last or alone in its 16-word
# block, and wave ranges long enough to cross frequency and image boundaries
# (the weight fragments held in registers must be replaced there).
NARROW_CASES = [
    # B, Cin, Cout, F, n
    (1, 1, 64, 3, 15),
    (1, 2, 7, 2, 16),
    (2, 3, 64, 5, 100),
    (1, 4, 130, 3, 47),
    (1, 5, 33, 4, 64),
    (2, 8, 64, 7, 31),
    (1, 9, 20, 3, 200),
    (1, 16, 96, 2, 70),
    (1, 3, 64, 1024, 255),
    (4, 3, 64, 256, 1024),
    (3, 7, 10, 600, 33),
]


@pytest.mark.parametrize("B,Cin,Cout,F,n", NARROW_CASES)
def test_homconv_narrow(ctx, orc, B, Cin, Cout, F, n):
    ct, w, r = _homconv_inputs(B, Cin, Cout, F, n, 41 * Cin + Cout + n)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("Cin", [3, 16])
def test_homconv_narrow_extreme_digits(ctx, orc, Cin):
    """Digits -128 and +127 against limbs -128, -127, 1 and p - 1 on the narrow kernel."""
    B, Cout, F, n = 2, 64, 3, 40
    ct = np.full((B, F, n + 1, Cin), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    ct[:, :, 1::2, : (Cin + 1) // 2] = 0x7F7F7F7F7F7F7F7F
    ct[:, :, ::5, :] = 2**64 - 1
    w = np.full((Cout, Cin, F), 0x8080, dtype=np.uint32)
    w[1::3] = P - 1
    r = np.full((B, Cout, F), P - 1, dtype=np.uint32)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


def test_homconv_extreme_words(ctx, orc):
    """All-ones words and W^ = p-1 maximise every limb sum."""
    B, Cin, Cout, F, n = 1, 70, 20, 2, 66
    ct = np.full((B, F, n + 1, Cin), 2**64 - 1, dtype=np.uint64)
    ct[:, :, ::3, :] = 2**63
    w = np.full((Cout, Cin, F), P - 1, dtype=np.uint32)
    r = np.full((B, Cout, F), P - 1, dtype=np.uint32)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("Cin", [169, 170, 300, 2048])
def test_homconv_extreme_digits(ctx, orc, Cin):
    """Every ciphertext digit -128 and W^ = 0x8080 (limbs -128, -127, 1): the
    largest same-sign shift sums, on both sides of the kernel's bound for its
    32-bit partial recombination (Cin <= 169)."""
    B, Cout, F, n = 1, 6, 2, 70
    ct = np.full((B, F, n + 1, Cin), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    ct[:, :, 1::2, : Cin // 2] = 0x7F7F7F7F7F7F7F7F  # every digit +127
    w = np.full((Cout, Cin, F), 0x8080, dtype=np.uint32)
    w[1] = P - 1
    r = np.full((B, Cout, F), 12345, dtype=np.uint32)
    ref = orc.homconv(ct, w, r, P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, ref)


# -------------------------------------------------------- argument checks ---


def test_degenerate_sizes_are_rejected_before_launch(ctx):
    from paper_2003_05328_amd.ensei import lib, _ptr

    L, h = lib(), ctx._h
    x = torch.zeros(64, dtype=torch.uint32, device="cuda:0")
    ct = torch.zeros(64, dtype=torch.uint64, device="cuda:0")
    s8 = torch.zeros(8, dtype=torch.int8, device="cuda:0")
    # empty batches, empty grids, zero channels, zero LWE dimension: ENSEI_ERR_ARG / SHAPE, nothing launched
    assert L.ensei_ntt2d(h, _ptr(x), _ptr(x), 0, 4, 4, None) == -1
    assert L.ensei_ntt2d(h, _ptr(x), _ptr(x), 1, 0, 4, None) == -2
    assert L.ensei_encrypt(h, _ptr(x), _ptr(s8), _ptr(x), 0, 1, 1, 8, 0, 0, _ptr(ct), None) == -1
    assert L.ensei_encrypt(h, _ptr(x), _ptr(s8), _ptr(x), 1, 1, 1, 0, 0, 0, _ptr(ct), None) == -1
    assert L.ensei_decrypt(h, _ptr(ct), _ptr(s8), 1, 0, 1, 8, _ptr(x), None) == -1
    assert L.ensei_homconv(h, _ptr(ct), _ptr(s8), _ptr(x), 1, 0, 4, 1, 4, _ptr(ct), None) == -1
    assert L.ensei_homconv(h, _ptr(ct), _ptr(s8), _ptr(x), 1, 4, 4, 1, 20000, _ptr(ct), None) == -6  # n > max
    torch.cuda.synchronize()


def test_binding_rejects_wrong_output_sizes(ctx):
    x = torch.zeros((3, 8, 8), dtype=torch.uint32, device="cuda:0")
    with pytest.raises(ValueError, match="elements"):
        ctx.ntt2d(x, out=torch.empty(3 * 64 - 1, dtype=torch.uint32, device="cuda:0"))
    with pytest.raises(ValueError, match="elements"):
        ctx.intt2d(x.view(3, 64), 8, 8, out=torch.empty(10, dtype=torch.uint32, device="cuda:0"))



def test_errors_are_reported(ctx):
    x = torch.zeros((2, 12, 16), dtype=torch.uint32, device="cuda:0")
    with pytest.raises(EnseiError, match="SHAPE"):
        ctx.ntt2d(x)
    big = torch.zeros((1, 1, 9, 4), dtype=torch.uint64, device="cuda:0")
    w1 = torch.zeros((4, 4, 1), dtype=torch.uint32, device="cuda:0")
    r1 = torch.zeros((1, 4, 1), dtype=torch.uint32, device="cuda:0")
    with pytest.raises(EnseiError, match="OVERLAP"):
        ctx.homconv_valu(big, w1, r1, out=big)
    s = torch.zeros(20000, dtype=torch.int8, device="cuda:0")
    m = torch.zeros(3, dtype=torch.uint32, device="cuda:0")
    e = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    with pytest.raises(EnseiError, match="LIMIT"):
        ctx.encrypt(m, s, e, 1)


# --------------------------------------------------- whole secure conv ------


def _gpu_round0(ctx, inp):
    S = inp.shape
    x = dev(inp.x)
    w = dev(inp.w)
    s = dev(inp.s)
    x_hat = ctx.ntt2d(x)  # [B][Cin][F]
    w_hat = ctx.weight_prep(w, S.H, S.W)
    pack = ctx.pack_weights(w_hat)
    ct_in = ctx.encrypt(x_hat, s, dev(inp.e), inp.seed_a)  # [B][F][n+1][Cin]
    r = dev(inp.r)
    ct_out = ctx.homconv(ct_in, pack, r, S.Cout)
    m = ctx.decrypt(ct_out, s)
    s_a = ctx.intt2d(m, S.H, S.W)
    s_b = ctx.server_share(r, S.H, S.W)
    return dict(x_hat=x_hat, w_hat=w_hat, ct_in=ct_in, ct_out=ct_out, m=m, s_a=s_a, s_b=s_b)


def test_small_secure_conv_bit_exact(ctx, orc):
    """16x16 grid, 3 -> 8 channels, n = 512: every intermediate equals the oracle's."""
    inp = synth.generate(configs.SMALL_16x16_3to8, P, seed=0)
    ref = orc.fdsc_round0(inp, P)
    got = _gpu_round0(ctx, inp)
    for k in ("x_hat", "w_hat", "ct_in", "ct_out", "m", "s_a", "s_b"):
        assert np.array_equal(host(got[k]), ref[k]), k
    y = (ref["s_a"].astype(np.int64) + ref["s_b"]) % P
    assert np.array_equal(y, orc.cyclic_conv(inp.x, inp.w, P))


FULL = [
    "conv16x16_c3to8_k3_n512",
    "conv32x32_c64to64_k3_n1024",
    "conv32x32_c64to64_k3_n1024_hidden",
    "conv64x64(56)_c64to64_k3_n1024",
    "conv128x128_c3to64_k7_n1024",
    "stack8_L1_32x32_c3to64",
    "stack8_L2_32x32_c64to64",
    "stack8_L3_16x16_c64to128",
    "stack8_L4_16x16_c128to128",
    "stack8_L5_8x8_c128to256",
    "stack8_L6_8x8_c256to256",
    "stack8_L7_4x4_c256to512",
    "stack8bin_L5_8x8_c128to256",
]


@pytest.mark.parametrize("name", FULL)
def test_full_size_layer(ctx, orc, name):
    S = configs.WORKLOADS[name]
    inp = synth.generate(S, P, seed=1)
    got = _gpu_round0(ctx, inp)
    # transforms: complete comparison
    x_hat = orc.ntt2d(inp.x, P).reshape(S.B, S.Cin, S.F)
    assert np.array_equal(host(got["x_hat"]), x_hat)
    w_hat = orc.weight_prep(inp.w, S.H, S.W, P)
    assert np.array_equal(host(got["w_hat"]), w_hat)
    # sampled ciphertext rows, each recomputed by the oracle from its own inputs
    g = np.random.default_rng(5)
    for _ in range(6):
        b, f = int(g.integers(S.B)), int(g.integers(S.F))
        cin = oracle_ct_in_rows(orc, x_hat, inp, b, f)
        for i in range(S.Cin):
            assert np.array_equal(ct_words(got["ct_in"], b, f, i), cin[i])
        for o in {0, S.Cout - 1, int(g.integers(S.Cout))}:
            ref_row = oracle_ct_out_row(orc, cin, w_hat, inp, b, o, f)
            assert np.array_equal(ct_words(got["ct_out"], b, f, o), ref_row)
            assert int(host(got["m"])[b, o, f]) == int(orc.decrypt(ref_row[None], inp.s, P)[0])
    # exact decryption everywhere: m = (sum_i W^ x^ + r) mod p
    # (products < 2^34, sums over Cin <= 512 stay below 2^43: exact in int64)
    exp_m = (np.einsum("oif,bif->bof", w_hat.astype(np.int64), x_hat.astype(np.int64)) + inp.r) % P
    assert np.array_equal(host(got["m"]).astype(np.int64), exp_m)
    # the two shares reconstruct the cyclic convolution
    y = (host(got["s_a"]).astype(np.int64) + host(got["s_b"])) % P
    assert np.array_equal(y, orc.cyclic_conv(inp.x, inp.w, P))


@pytest.mark.parametrize("name", ["conv32x32_c64to64_k3_n1024", "conv64x64(56)_c64to64_k3_n1024"])
def test_full_size_ciphertexts_elementwise(ctx, orc, name):
    """At full size, every word of ct_in and of ct_out equals the oracle's
    (its Enc and HomConv over the whole layer), with the exact decryptions."""
    S = configs.WORKLOADS[name]
    inp = synth.generate(S, P, seed=2)
    got = _gpu_round0(ctx, inp)
    x_hat = orc.ntt2d(inp.x, P).reshape(S.B, S.Cin, S.F)
    w_hat = orc.weight_prep(inp.w, S.H, S.W, P)
    ct_in = orc.encrypt(x_hat, inp.s, inp.e, inp.seed_a, P)
    assert np.array_equal(host(got["ct_in"]), ct_in)
    del got["ct_in"]
    ct_out = orc.homconv(ct_in, w_hat, inp.r, P)
    del ct_in
    assert np.array_equal(host(got["ct_out"]), ct_out)
    assert np.array_equal(host(got["m"]), orc.decrypt(ct_out, inp.s, P))
