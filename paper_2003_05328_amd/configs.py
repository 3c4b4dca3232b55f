"""Workload shapes of the secure-convolution hot path.

Every workload is a cyclic H x W grid, Cin -> Cout channels, a kh x kw filter,
LWE dimension n, modulus p = 65537 for transform, shares and plaintext, and
ciphertext modulus 2^64. Shapes follow the paper's CIFAR-10 / ImageNet-style
layers (Appendix B networks) at the sizes fixed for this build.
"""
from __future__ import annotations

from .synth import LayerShape

P = 65537

# Small single secure conv: 16x16 grid, 3 -> 8 channels, 3x3, n = 512.
SMALL_16x16_3to8 = LayerShape(H=16, W=16, Cin=3, Cout=8, kh=3, kw=3, n=512)

# CIFAR-shaped layer: 32x32 grid, 64 -> 64 channels, 3x3, n = 1024 (the bench workload).
CIFAR_32x32_64to64 = LayerShape(H=32, W=32, Cin=64, Cout=64, kh=3, kw=3, n=1024)
CIFAR_32x32_64to64_HIDDEN = LayerShape(H=32, W=32, Cin=64, Cout=64, kh=3, kw=3, n=1024, hidden=True)

# Seven-layer 3x3 stack, batch of 8 images (each layer an independent secure conv).
STACK_LAYERS = [
    (3, 64, 32),
    (64, 64, 32),
    (64, 128, 16),
    (128, 128, 16),
    (128, 256, 8),
    (256, 256, 8),
    (256, 512, 4),
]


def stack_shapes(binary: bool = False, B: int = 8) -> list[LayerShape]:
    """The stack's layers: pixels in [0, 255] into the first, residues
    uniform in [0, p) (hidden activations) into the others."""
    return [
        LayerShape(H=hw, W=hw, Cin=ci, Cout=co, kh=3, kw=3, n=1024, B=B, binary=binary, hidden=k > 0)
        for k, (ci, co, hw) in enumerate(STACK_LAYERS)
    ]


# ImageNet-shaped large layers.
IMAGENET_64x64_56_64to64 = LayerShape(H=64, W=64, Cin=64, Cout=64, kh=3, kw=3, n=1024, img_h=56, img_w=56)
IMAGENET_128x128_3to64_7x7 = LayerShape(H=128, W=128, Cin=3, Cout=64, kh=7, kw=7, n=1024)

WORKLOADS = {
    "conv16x16_c3to8_k3_n512": SMALL_16x16_3to8,
    "conv32x32_c64to64_k3_n1024": CIFAR_32x32_64to64,
    "conv32x32_c64to64_k3_n1024_hidden": CIFAR_32x32_64to64_HIDDEN,
    "conv64x64(56)_c64to64_k3_n1024": IMAGENET_64x64_56_64to64,
    "conv128x128_c3to64_k7_n1024": IMAGENET_128x128_3to64_7x7,
}
for _i, _s in enumerate(stack_shapes()):
    WORKLOADS[f"stack8_L{_i + 1}_{_s.H}x{_s.W}_c{_s.Cin}to{_s.Cout}"] = _s
for _i, _s in enumerate(stack_shapes(binary=True)):
    WORKLOADS[f"stack8bin_L{_i + 1}_{_s.H}x{_s.W}_c{_s.Cin}to{_s.Cout}"] = _s


# The packed (BFV / RLWE) instantiation's parameter sets: t = p_E and
# ceil(lg q) of Table 2 (ENSEI-NTT), n = 2048; q = q0 q1, two primes
# = 1 mod 2n, the limbs with the smallest centred q mod t among those of the
# stated bit length (the same rule the checker's golden file records).
PACKED_SETS = {
    "binary": dict(t=12289, q0=8380417, q1=4005889, n=2048),
    "medium": dict(t=147457, q0=134176769, q1=63062017, n=2048),
    "high": dict(t=2363393, q0=1073692673, q1=561770497, n=2048),
}
