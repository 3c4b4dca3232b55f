"""Pure-Python big-integer brute force on tiny inputs (test helper).

Independent of the C oracle: everything here is computed with Python's
arbitrary-precision integers, straight from the definitions, with no
modular tricks and no fixed-width arithmetic.
"""
from __future__ import annotations

M64 = 1 << 64


def brute_root(p: int, N: int, inverse: bool = False) -> int:
    """An element of order exactly N found by search (not by formula)."""
    # smallest generator g by brute force over the group order
    order = p - 1
    for g in range(2, p):
        x, k = g, 1
        while x != 1:
            x = x * g % p
            k += 1
        if k == order:
            break
    w = pow(g, order // N, p)
    return pow(w, -1, p) if inverse else w


def brute_dft2d(x, p: int, inverse: bool = False):
    """x: list of H lists of W ints -> 2D DFT over Z_p (double sum)."""
    H, W = len(x), len(x[0])
    wH, wW = brute_root(p, H, inverse), brute_root(p, W, inverse)
    sc = pow(H * W, -1, p) if inverse else 1
    return [
        [
            sc * sum(x[i1][i2] * pow(wH, i1 * k1, p) * pow(wW, i2 * k2, p) for i1 in range(H) for i2 in range(W)) % p
            for k2 in range(W)
        ]
        for k1 in range(H)
    ]


def brute_cyclic_conv(x, w, p: int):
    """Single channel: x H x W, w kh x kw (signed ints) -> cyclic conv mod p."""
    H, W = len(x), len(x[0])
    kh, kw = len(w), len(w[0])
    return [
        [
            sum(w[j1][j2] * x[(m1 - j1) % H][(m2 - j2) % W] for j1 in range(kh) for j2 in range(kw)) % p
            for m2 in range(W)
        ]
        for m1 in range(H)
    ]


GAMMA = 0x9E3779B97F4A7C15


def splitmix64_stream(seed: int, count: int):
    """The first `count` outputs of a stateful SplitMix64 generator."""
    state = seed % M64
    out = []
    for _ in range(count):
        state = (state + GAMMA) % M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % M64
        out.append(z ^ (z >> 31))
    return out


def brute_delta(p: int) -> int:
    return M64 // p


def brute_decode(phi: int, p: int) -> int:
    """Round(p * phi / 2^64) mod p with exact rationals: nearest integer, ties up."""
    from fractions import Fraction

    v = Fraction(phi * p, M64)
    q = int(v)  # floor for non-negative
    if v - q >= Fraction(1, 2):
        q += 1
    return q % p
