"""Seeded synthetic inputs for one frequency-domain secure convolution (FDSC).

This module only draws random numbers; it holds none of the method's
arithmetic (no transform, no modular reduction, no encryption). Both the CPU
oracle tests and the GPU path read the arrays it returns, so the two sides see
bit-identical inputs.

Draw order (fixed, from one seed, numpy PCG64 seeded through SeedSequence):

1. image pixels ``x_img`` [B][Cin][h][w]: uniform ints in [0, 255] for a first
   layer, or uniform in [0, p) for a hidden layer (inputs that are already
   residues of an earlier layer's shares);
2. filters ``w`` [Cout][Cin][kh][kw] int32: uniform ints in [-8, 8], or uniform
   in {-1, +1} for the binary-weight variant (BinaryConnect-style weights,
   Sec. 5.2 of the paper);
3. secret key ``s`` [n] int8: i.i.d. uniform ternary {-1, 0, 1}, one key per
   client (the batch of images belongs to one client);
4. encryption errors ``e`` [B][Cin][H*W] int32: rounded Gaussian with
   sigma = 3.2, sampled on the host so no floating-point sampler has to agree
   bit-for-bit across devices;
5. server masks ``r`` [B][Cout][H*W] uint32: uniform in [0, p) (the server's
   frequency-domain share is -r mod p; HomShare, Eq. (homshare));
6. ``seed_a``: one uint64 that keys the counter-based generator both sides
   implement for the uniform LWE a-vectors.

The image is placed at the top-left of an H x W grid of zeros (the padding
step of the protocol, Sec. 4.1); when h == H and w == W it fills the grid.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SIGMA = 3.2


@dataclass(frozen=True)
class LayerShape:
    """One secure-convolution layer: grid, channels, filter, LWE dimension."""

    H: int
    W: int
    Cin: int
    Cout: int
    kh: int
    kw: int
    n: int
    B: int = 1
    img_h: int | None = None  # image region placed top-left; None = full grid
    img_w: int | None = None
    hidden: bool = False  # inputs uniform in [0, p) instead of pixels
    binary: bool = False  # filters in {-1, +1}

    @property
    def F(self) -> int:
        return self.H * self.W

    @property
    def ih(self) -> int:
        return self.H if self.img_h is None else self.img_h

    @property
    def iw(self) -> int:
        return self.W if self.img_w is None else self.img_w


@dataclass
class LayerInputs:
    shape: LayerShape
    p: int
    x: np.ndarray  # uint32 [B][Cin][H][W], zero-padded image
    w: np.ndarray  # int32 [Cout][Cin][kh][kw]
    s: np.ndarray  # int8 [n]
    e: np.ndarray  # int32 [B][Cin][F]
    r: np.ndarray  # uint32 [B][Cout][F]
    seed_a: int  # uint64 key of the a-vector generator


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def generate(shape: LayerShape, p: int, seed: int) -> LayerInputs:
    """Draw every input of one layer from ``seed`` in the documented order."""
    g = rng_for(seed)
    S = shape
    if S.hidden:
        img = g.integers(0, p, size=(S.B, S.Cin, S.ih, S.iw), dtype=np.int64)
    else:
        img = g.integers(0, 256, size=(S.B, S.Cin, S.ih, S.iw), dtype=np.int64)
    x = np.zeros((S.B, S.Cin, S.H, S.W), dtype=np.uint32)
    x[:, :, : S.ih, : S.iw] = img.astype(np.uint32)
    if S.binary:
        w = (2 * g.integers(0, 2, size=(S.Cout, S.Cin, S.kh, S.kw), dtype=np.int64) - 1).astype(np.int32)
    else:
        w = g.integers(-8, 9, size=(S.Cout, S.Cin, S.kh, S.kw), dtype=np.int64).astype(np.int32)
    s = g.integers(-1, 2, size=(S.n,), dtype=np.int64).astype(np.int8)
    e = np.rint(g.normal(0.0, SIGMA, size=(S.B, S.Cin, S.F))).astype(np.int32)
    r = g.integers(0, p, size=(S.B, S.Cout, S.F), dtype=np.int64).astype(np.uint32)
    seed_a = int(g.integers(0, 2**64, dtype=np.uint64))
    return LayerInputs(S, p, x, w, s, e, r, seed_a)


def uniform_u32(seed: int, shape, hi: int) -> np.ndarray:
    """Uniform uint32 array in [0, hi) (for transform-only tests and benches)."""
    return rng_for(seed).integers(0, hi, size=shape, dtype=np.int64).astype(np.uint32)


def uniform_u64(seed: int, shape) -> np.ndarray:
    """Uniform uint64 words (stand-in ciphertexts for HomConv-only tests)."""
    return rng_for(seed).integers(0, 2**64, size=shape, dtype=np.uint64)


def ternary(seed: int, n: int) -> np.ndarray:
    return rng_for(seed).integers(-1, 2, size=(n,), dtype=np.int64).astype(np.int8)


def rounded_gaussian(seed: int, shape) -> np.ndarray:
    return np.rint(rng_for(seed).normal(0.0, SIGMA, size=shape)).astype(np.int32)
