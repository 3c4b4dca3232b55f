"""GPU parity of the device error sampler (the rounded Gaussian of sigma 3.2
drawn from the public generator): the library's thresholds against the
oracle's, every draw against the oracle bit for bit, and encryption with
device-drawn errors decrypting exactly."""
import math

import numpy as np
import pytest

import oracle
from paper_2003_05328_amd import synth
from paper_2003_05328_amd.ensei import Context
from tests.gpu_helpers import P, dev, host

pytestmark = pytest.mark.gpu


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


def test_error_table_matches_oracle(ctx):
    # the library computes its thresholds in long double, the oracle in
    # 80-digit decimal arithmetic; the draws agree only if these agree
    assert ctx.error_table() == oracle.cdt_table()


@pytest.mark.parametrize("B,C,F,idx0", [(1, 1, 1, 0), (2, 3, 5, 9), (1, 64, 1024, 0), (3, 70, 33, 2**64 - 100),
                                        (8, 3, 1024, 12345)])
def test_sample_errors(ctx, orc, B, C, F, idx0):
    seed_e = 0x5EED0000 + B * 1000 + C
    got = host(ctx.sample_errors(seed_e, B, C, F, ct_index0=idx0))
    assert np.array_equal(got, orc.sample_errors(seed_e, B, C, F, ct_index0=idx0))


def test_sample_errors_distribution(ctx):
    N = 1 << 22
    x = host(ctx.sample_errors(2024, 1, 1, N)).astype(np.float64).ravel()
    sigma = oracle.SIGMA_NUM / oracle.SIGMA_DEN
    var = sigma**2 + 1 / 12
    assert abs(x.mean()) < 4 * math.sqrt(var / N)
    assert abs(x.var() / var - 1) < 0.005
    for k in range(6):  # P(|e| = k) against the rounded Gaussian's
        pk = math.erf((k + 0.5) / (sigma * math.sqrt(2))) - (math.erf((k - 0.5) / (sigma * math.sqrt(2))) if k else 0)
        assert abs((np.abs(x) == k).mean() - pk) < 5 * math.sqrt(pk * (1 - pk) / N), k


def test_encrypt_with_device_errors(ctx, orc):
    """Enc with device-drawn errors: the words equal the oracle's Enc with the
    oracle's draws, and decryption is exact."""
    B, C, F, n = 2, 64, 16, 256
    m = synth.uniform_u32(130, (B, C, F), P)
    s = synth.ternary(131, n)
    seed_a, seed_e = 0xABCDEF, 0x123456
    e = ctx.sample_errors(seed_e, B, C, F)
    ct = ctx.encrypt(dev(m), dev(s), e, seed_a)
    ref = orc.encrypt(m, s, orc.sample_errors(seed_e, B, C, F), seed_a, P)
    assert np.array_equal(host(ct), ref)
    assert np.array_equal(host(ctx.decrypt(ct, dev(s))), m)


def test_sample_errors_argument_errors(ctx):
    from paper_2003_05328_amd.ensei import _ptr, lib

    L, h, st = lib(), ctx._h, ctx._stream()
    e = dev(np.zeros(8, dtype=np.int32))
    assert L.ensei_sample_errors(h, 1, 0, 1, 1, 8, None, st) == -1
    assert L.ensei_sample_errors(h, 1, 0, 0, 1, 8, _ptr(e), st) == -1
    assert L.ensei_sample_errors(h, 1, 0, 1, 1, 1, e.data_ptr() + 2, st) == -4
    assert L.ensei_sample_errors(h, 1, 0, 1 << 30, 1 << 10, 1 << 10, _ptr(e), st) == -6  # beyond 2^40 errors
    assert L.ensei_error_table(h, None, 32) == -1
    assert not host(e).any()
