"""GPU parity at the ABI's maximum sizes: the largest LWE dimension (Enc, Dec,
HomConv and its seeded form), the largest input channel count (the bound
that keeps the matrix cores' i32 limb sums exact, with the digits that make
those sums largest) and the largest output channel count, each against the
oracle, and one step past each limit refused."""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05328_amd import synth
from paper_2003_05328_amd.ensei import Context, EnseiError
from tests.gpu_helpers import P, dev, host

pytestmark = pytest.mark.gpu

MAX_N, MAX_CIN, MAX_COUT = 16384, 32768, 65536


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


def test_largest_lwe_dimension(ctx, orc):
    B, C, F, n = 1, 64, 2, MAX_N
    m = synth.uniform_u32(500, (B, C, F), P)
    s = synth.ternary(501, n)
    e = synth.rounded_gaussian(502, (B, C, F))
    ct = ctx.encrypt(dev(m), dev(s), dev(e), 5)
    ref = orc.encrypt(m, s, e, 5, P)
    assert np.array_equal(host(ct), ref)
    assert np.array_equal(host(ctx.decrypt(ct, dev(s))), m)
    Cout = 64
    w = synth.uniform_u32(503, (Cout, C, F), P)
    r = synth.uniform_u32(504, (B, Cout, F), P)
    pack = ctx.pack_weights(dev(w))
    out = ctx.homconv(ct, pack, dev(r), Cout)
    ref_out = orc.homconv(ref, w, r, P)
    assert np.array_equal(host(out), ref_out)
    bw = ctx.encrypt_seeded(dev(m), dev(s), dev(e), 5)
    assert np.array_equal(host(ctx.homconv_seeded(bw, n, 5, pack, dev(r), Cout)), ref_out)
    with pytest.raises(EnseiError, match="LIMIT"):
        ctx.encrypt(dev(m), dev(synth.ternary(505, n + 1)), dev(e), 5)


def test_largest_input_channel_count(ctx, orc):
    """Cin = 32768: every shift sum reaches its largest magnitude (digits -128
    and +127 against the limbs of 0x8080 and p - 1), 512 K steps."""
    B, Cin, Cout, F, n = 1, MAX_CIN, 2, 1, 8
    ct = np.full((B, F, n + 1, Cin), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    ct[:, :, 1::2, : Cin // 2] = 0x7F7F7F7F7F7F7F7F
    w = np.full((Cout, Cin, F), 0x8080, dtype=np.uint32)
    w[1, ::3, :] = P - 1
    r = np.full((B, Cout, F), P - 1, dtype=np.uint32)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, orc.homconv(ct, w, r, P))
    w2 = dev(np.zeros((Cout, Cin + 1, F), dtype=np.uint32))
    with pytest.raises(EnseiError, match="LIMIT"):
        ctx.pack_weights(w2)


def test_largest_output_channel_count(ctx, orc):
    """Cout = 65536 (1024 row tiles) on the narrow-input kernel."""
    B, Cin, Cout, F, n = 1, 1, MAX_COUT, 1, 4
    ct = synth.uniform_u64(510, (B, F, n + 1, Cin))
    w = synth.uniform_u32(511, (Cout, Cin, F), P)
    r = synth.uniform_u32(512, (B, Cout, F), P)
    got = host(ctx.homconv(dev(ct), ctx.pack_weights(dev(w)), dev(r), Cout))
    assert np.array_equal(got, orc.homconv(ct, w, r, P))
    w2 = dev(np.zeros((Cout + 1, Cin, F), dtype=np.uint32))
    with pytest.raises(EnseiError, match="LIMIT"):
        ctx.pack_weights(w2)
    torch.cuda.synchronize()
