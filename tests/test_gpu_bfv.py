"""GPU parity of the packed (BFV / RLWE) instantiation against its oracle
(oracle/bfv.py): every call bit for bit under Table 2's three parameter sets
(n = 2048) and toy sets (n = 64, 128, 1024, 4096), packings with several channels per
vector (and a partial last one), one channel per vector and channels
spanning two vectors; the whole packed secure convolution, whose shares add
up to the cyclic convolution mod t; and argument errors."""
import numpy as np
import pytest
import torch

import oracle
from oracle import bfv as obfv
from paper_2003_05328_amd.ensei import Context, EnseiError
from paper_2003_05328_amd.ensei_bfv import BfvContext, geometry
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

SETS = dict(obfv.table2_params())
SETS["toy"] = obfv.Params("toy", 257, 1073692673, 561770497, 64)
# ring degrees whose transforms end in a one-stage pass (n = 128, 1024: the
# stages go three at a time) and that give a thread two units per pass
# (n = 4096); primes below 2^30, each 1 mod 2n
SETS["toy128"] = obfv.Params("toy128", 257, 1073692673, 561770497, 128)
SETS["toy1024"] = obfv.Params("toy1024", 12289, 1073692673, 561770497, 1024)
SETS["toy4096"] = obfv.Params("toy4096", 40961, 1073692673, 536813569, 4096)


@pytest.fixture(scope="module")
def orc():
    o = obfv.default()
    o.set_threads(16)
    return o


@pytest.fixture(scope="module", params=sorted(SETS))
def pr_ctx(request):
    pr = SETS[request.param]
    c = BfvContext(pr.t, pr.q0, pr.q1, pr.n, 0)
    yield pr, c
    c.close()


def _key(pr, seed):
    g = np.random.default_rng(seed)
    return g.integers(-1, 2, size=pr.n).astype(np.int8)


def test_key(orc, pr_ctx):
    pr, c = pr_ctx
    s = _key(pr, 1)
    got = host(c.key(dev(s)))
    ref = orc.key(pr, s)
    assert np.array_equal(got[:, 0], ref)
    for l, m in enumerate((pr.q0, pr.q1)):
        assert np.array_equal(got[l, 1].astype(np.uint64), (ref[l].astype(np.uint64) << np.uint64(32)) // np.uint64(m))


def _shapes(pr):
    n = pr.n
    return [(2, 5, n // 4), (1, 3, n), (1, 2, 2 * n), (1, 1, n // 16)]


def test_encrypt(orc, pr_ctx):
    pr, c = pr_ctx
    s = _key(pr, 2)
    s_hat = c.key(dev(s))
    for k, (B, C_, F) in enumerate(_shapes(pr)):
        g = np.random.default_rng(10 + k)
        x = g.integers(0, pr.t, size=(B, C_, F)).astype(np.uint32)
        x[0, 0, :3] = [0, pr.t - 1, pr.t // 2]
        nv = B * c.vectors(C_, F)
        e = np.rint(g.normal(0, 4.0, size=(nv, pr.n))).astype(np.int32)
        e[0, :2] = [-40, 40]
        got = host(c.encrypt(dev(x), s_hat, dev(e), seed_a=77, ct_index0=5))
        ref = orc.encrypt(pr, orc.pack(x, pr.n).reshape(nv, pr.n), s, e, 77, ct_index0=5)
        assert np.array_equal(got, ref), (B, C_, F)


def test_encode_filters_and_masks(orc, pr_ctx):
    pr, c = pr_ctx
    for k, (Cout, Cin, F) in enumerate([(3, 5, pr.n // 4), (2, 2, 2 * pr.n)]):
        g = np.random.default_rng(20 + k)
        w = g.integers(0, pr.t, size=(Cout, Cin, F)).astype(np.uint32)
        w[0, 0, :2] = [pr.t - 1, pr.t // 2 + 1]
        got = host(c.encode_filters(dev(w)))
        ref = orc.filters(pr, w)  # [Cout][G][K][L][n]
        assert np.array_equal(got[..., 0, :], ref)
        for l, m in enumerate((pr.q0, pr.q1)):
            comp = (ref[..., l, :].astype(np.uint64) << np.uint64(32)) // np.uint64(m)
            assert np.array_equal(got[..., l, 1, :].astype(np.uint64), comp)
    g = np.random.default_rng(29)
    r = g.integers(0, pr.t, size=(3, pr.n)).astype(np.uint32)
    assert np.array_equal(host(c.encode_masks(dev(r))), orc.encode(pr, r, scaled=True))


def test_homconv(orc, pr_ctx):
    pr, c = pr_ctx
    # G = 2 and 3 input vectors, and 20 (exact 64-bit sums of 16 products, then of 4)
    for k, (B, Cin, Cout, F) in enumerate([(2, 5, 6, pr.n // 4), (1, 3, 2, pr.n), (1, 2, 5, 2 * pr.n),
                                           (1, 20, 3, pr.n)]):
        g = np.random.default_rng(30 + k)
        P, K, G = geometry(Cin, F, pr.n)
        ct = np.stack([g.integers(0, m, size=(B * G * K, 2, pr.n)) for m in (pr.q0, pr.q1)], axis=1).astype(np.uint32)
        w = g.integers(0, pr.t, size=(Cout, Cin, F)).astype(np.uint32)
        w_enc = c.encode_filters(dev(w))
        mask = np.stack([g.integers(0, m, size=(B * Cout * K, pr.n)) for m in (pr.q0, pr.q1)], axis=1).astype(np.uint32)
        got = host(c.homconv(dev(ct), w_enc, dev(mask), B, Cin, F))
        ref = orc.homconv(pr, ct.reshape(B, G * K, 2, 2, pr.n), orc.filters(pr, w), mask.reshape(B, Cout * K, 2, pr.n))
        assert np.array_equal(got, ref.reshape(got.shape)), (B, Cin, Cout, F)


def test_decrypt(orc, pr_ctx):
    pr, c = pr_ctx
    s = _key(pr, 3)
    s_hat = c.key(dev(s))
    g = np.random.default_rng(40)
    # fresh encryptions, and arbitrary words (every rounding case of random phases)
    v = g.integers(0, pr.t, size=(3, pr.n)).astype(np.uint32)
    ct = orc.encrypt(pr, v, s, np.rint(g.normal(0, 4.0, size=v.shape)).astype(np.int32), 9)
    rnd = np.stack([g.integers(0, m, size=(4, 2, pr.n)) for m in (pr.q0, pr.q1)], axis=1).astype(np.uint32)
    for words in (ct, rnd):
        got = host(c.decrypt(dev(words), s_hat))
        assert np.array_equal(got, orc.decrypt(pr, words, s))
    assert np.array_equal(host(c.decrypt(dev(ct), s_hat)), v)


def test_fold(orc, pr_ctx):
    pr, c = pr_ctx
    g = np.random.default_rng(50)
    for B, C_, F in ((2, 3, pr.n // 8), (1, 2, pr.n), (1, 3, 2 * pr.n)):
        P, K, G = geometry(1, F, pr.n)
        v = g.integers(0, pr.t, size=(B, C_ * K, pr.n)).astype(np.uint32)
        y = orc.fold(pr, v, F)
        assert np.array_equal(host(c.fold(dev(v.reshape(-1, pr.n)), B, C_, F)), y)
        assert np.array_equal(host(c.fold(dev(v.reshape(-1, pr.n)), B, C_, F, negate=True)), (pr.t - y) % pr.t)


def test_rerandomize(orc, pr_ctx):
    """Circuit privacy: the GPU's re-randomisation equals the oracle's, word
    for word, and leaves the decryption unchanged."""
    pr, c = pr_ctx
    g = np.random.default_rng(55)
    s = _key(pr, 56)
    s_hat = c.key(dev(s))
    e_pk = np.rint(g.normal(0, 4.0, size=(1, pr.n))).astype(np.int32)
    pk = c.encrypt(dev(np.zeros((1, 1, pr.n), np.uint32)), s_hat, dev(e_pk), seed_a=57)
    ref_pk = orc.encrypt(pr, np.zeros((1, pr.n), np.int64), s, e_pk, 57)
    assert np.array_equal(host(pk), ref_pk)
    v = g.integers(0, pr.t, size=(3, pr.n)).astype(np.uint32)
    ct = orc.encrypt(pr, v, s, np.rint(g.normal(0, 4.0, size=v.shape)).astype(np.int32), 58)
    flood = min(pr.delta // 16, 2**30)
    got = c.rerandomize(dev(ct), pk[0], seed_r=59, flood=flood, ct_index0=11)
    ref = orc.rerandomize(pr, ct, ref_pk[0], 59, flood, ct_index0=11)
    assert np.array_equal(host(got), ref)
    assert np.array_equal(host(c.decrypt(got, s_hat)), v)
    with pytest.raises(EnseiError, match="ARG"):
        c.rerandomize(got, pk[0], 1, 2**31)


@pytest.mark.parametrize("name", ["binary", "high", "toy"])
def test_packed_secure_conv(orc, name):
    """The whole packed start round on the GPU: NTT2D mod t, Enc, filters,
    masks, HomConv, Dec, fold, INTT2D, and the server's share; every
    intermediate equals the oracle's and the shares add up to x (*) w mod t."""
    pr = SETS[name]
    H = W = 32 if pr.n >= 1024 else 8
    B, Cin, Cout, kh = 2, 5, 3, 3
    F = H * W
    c = BfvContext(pr.t, pr.q0, pr.q1, pr.n, 0)
    lwe = Context(pr.t, 0)
    lorc = oracle.default()
    g = np.random.default_rng(60)
    x = g.integers(0, 256, size=(B, Cin, H, W)).astype(np.uint32)
    w = g.integers(-8, 9, size=(Cout, Cin, kh, kh)).astype(np.int32)
    s = _key(pr, 61)
    P, K, G = geometry(Cin, F, pr.n)
    e = np.rint(g.normal(0, 4.0, size=(B * G * K, pr.n))).astype(np.int32)
    r = g.integers(0, pr.t, size=(B * Cout * K, pr.n)).astype(np.uint32)
    # client
    x_hat = lwe.ntt2d(dev(x)).view(B, Cin, F)
    s_hat = c.key(dev(s))
    ct_in = c.encrypt(x_hat, s_hat, dev(e), seed_a=123)
    # server
    w_hat = lwe.weight_prep(dev(w), H, W)
    w_enc = c.encode_filters(w_hat)
    ct_out = c.homconv(ct_in, w_enc, c.encode_masks(dev(r)), B, Cin, F)
    s_b = lwe.intt2d(c.fold(dev(r), B, Cout, F, negate=True).view(B * Cout, F), H, W)
    # client
    y = c.fold(c.decrypt(ct_out, s_hat), B, Cout, F)
    s_a = lwe.intt2d(y.view(B * Cout, F), H, W)
    torch.cuda.synchronize()
    ref = orc.secure_conv(pr, lorc.ntt2d(x, pr.t).reshape(B, Cin, F), lorc.weight_prep(w, H, W, pr.t),
                          r.reshape(B, Cout * K, pr.n), s, e.reshape(B, G * K, pr.n), 123)
    assert np.array_equal(host(ct_in), ref["ct_in"].reshape(-1, 2, 2, pr.n))
    assert np.array_equal(host(ct_out), ref["ct_out"].reshape(-1, 2, 2, pr.n))
    assert np.array_equal(host(y), ref["y"])
    conv = lorc.cyclic_conv(x, w, pr.t)
    shares = (host(s_a).astype(np.int64).reshape(B, Cout, H, W) + host(s_b).reshape(B, Cout, H, W)) % pr.t
    assert np.array_equal(shares, conv)
    c.close()
    lwe.close()


def test_errors(pr_ctx):
    pr, c = pr_ctx
    with pytest.raises(EnseiError, match="MODULUS"):
        BfvContext(pr.t, pr.q0, pr.q0, pr.n, 0)
    with pytest.raises(EnseiError, match="MODULUS"):
        BfvContext(12289, 8380417, 4005889, 4096, 0)  # 2n = 8192 does not divide 12288
    with pytest.raises(EnseiError, match="ARG"):
        BfvContext(pr.t, pr.q0, pr.q1, 48, 0)
    x = torch.zeros((1, 1, 3 * 8), dtype=torch.uint32, device="cuda:0")  # F = 24: not a power of two
    s_hat = torch.zeros((2, 2, pr.n), dtype=torch.uint32, device="cuda:0")
    with pytest.raises(EnseiError, match="SHAPE"):
        c._call("ensei_bfv_encrypt", x.data_ptr(), 1, 1, 24, s_hat.data_ptr(), s_hat.data_ptr(), 0, 0, s_hat.data_ptr())
    ct = torch.zeros((1, 2, 2, pr.n), dtype=torch.uint32, device="cuda:0")
    with pytest.raises(EnseiError, match="OVERLAP"):
        c._call("ensei_bfv_decrypt", ct.data_ptr(), s_hat.data_ptr(), 1, ct.data_ptr())
