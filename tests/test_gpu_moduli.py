"""GPU parity with the paper's own plaintext moduli (Table 2's p_E for the
Binary, Medium and High parameter sets, tests/golden/table2_moduli.txt): the
whole step (NTT2D, weight preparation, Enc, HomConv, Dec, INTT2D, the
server's share) against the oracle, every intermediate bit for bit, on the
narrow, folded, paired and deep HomConv kernels.

For p other than 65537, Delta p = 2^64 - rho with rho = 2^64 mod p > 1, so each
wrap of the plaintext past p inside HomConv adds -rho to the noise. The shares
reconstruct the convolution when Cin p rho stays below Delta / 4 (a margin
over the Delta / 2 decoding bound). That holds for the Binary and Medium
moduli at these sizes but not for the High one, which gets parity only.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2003_05328_amd import synth
from paper_2003_05328_amd.ensei import Context
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_moduli.txt")


def _table2_pe():
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, _pn, pe, _lgq, _n = line.split()
                out.append((name, int(pe)))
    return out


MODULI = _table2_pe()

SHAPES = [
    # narrow HomConv (Cin <= 8)
    synth.LayerShape(H=16, W=16, Cin=3, Cout=8, kh=3, kw=3, n=64, B=2),
    # folded streaming HomConv
    synth.LayerShape(H=4, W=8, Cin=17, Cout=5, kh=3, kw=2, n=33, B=3, hidden=True),
    # paired streaming HomConv, two row tiles
    synth.LayerShape(H=8, W=8, Cin=64, Cout=70, kh=3, kw=3, n=100, B=1, hidden=True),
    # deep HomConv (three row tiles, three K steps)
    synth.LayerShape(H=4, W=4, Cin=130, Cout=130, kh=3, kw=3, n=33, B=1, hidden=True),
]


@pytest.fixture(scope="module")
def orc():
    o = oracle.default()
    o.set_threads(16)
    return o


@pytest.fixture(scope="module", params=[pe for _, pe in MODULI], ids=[name for name, _ in MODULI])
def pctx(request):
    c = Context(request.param, 0)
    yield request.param, c
    c.close()


@pytest.mark.parametrize("k", range(len(SHAPES)))
def test_step_with_table2_modulus(orc, pctx, k):
    p, ctx = pctx
    S = SHAPES[k]
    inp = synth.generate(S, p, 300 + k)
    ref = orc.fdsc_round0(inp, p)
    x_hat = ctx.ntt2d(dev(inp.x))
    assert np.array_equal(host(x_hat), ref["x_hat"].reshape(S.B, S.Cin, S.F))
    w_hat = ctx.weight_prep(dev(inp.w), S.H, S.W)
    assert np.array_equal(host(w_hat), ref["w_hat"])
    s, e, r = dev(inp.s), dev(inp.e), dev(inp.r)
    ct_in = ctx.encrypt(x_hat, s, e, inp.seed_a)
    assert np.array_equal(host(ct_in), ref["ct_in"])
    ct_out = ctx.homconv(ct_in, ctx.pack_weights(w_hat), r, S.Cout)
    assert np.array_equal(host(ct_out), ref["ct_out"])
    m = ctx.decrypt(ct_out, s)
    assert np.array_equal(host(m), ref["m"])
    s_a = ctx.intt2d(m, S.H, S.W)
    assert np.array_equal(host(s_a), ref["s_a"].reshape(S.B, S.Cout, S.H, S.W))
    s_b = ctx.server_share(r, S.H, S.W)
    assert np.array_equal(host(s_b), ref["s_b"].reshape(S.B, S.Cout, S.H, S.W))
    # the shares reconstruct the convolution where the wrap noise fits
    rho, delta = 2**64 % p, 2**64 // p
    if S.Cin * p * rho < delta // 4:
        conv = orc.cyclic_conv(inp.x, inp.w, p)
        y = (host(s_a).astype(np.int64) + host(s_b)) % p
        assert np.array_equal(y, conv.astype(np.int64))


def test_fresh_ciphertexts_decrypt_under_every_modulus(orc):
    """Enc then Dec is the identity for every Table 2 modulus (no HomConv, so
    no wrap noise), at the extreme plaintexts 0, 1, p - 1."""
    for _, p in MODULI:
        ctx = Context(p, 0)
        try:
            B, C, F, n = 1, 5, 7, 64
            m = synth.uniform_u32(400, (B, C, F), p)
            m.flat[:3] = [0, 1, p - 1]
            s = synth.ternary(401, n)
            e = synth.rounded_gaussian(402, (B, C, F))
            ct = ctx.encrypt(dev(m), dev(s), dev(e), 77)
            assert np.array_equal(host(ct), orc.encrypt(m, s, e, 77, p))
            assert np.array_equal(host(ctx.decrypt(ct, dev(s))), m)
        finally:
            ctx.close()
