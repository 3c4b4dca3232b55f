"""Writes tests/golden/bfv_params.txt: the packed instantiation's parameter
sets, from Table 2 (ENSEI-NTT: p_E and ceil(lg q), n = 2048) and the limb
rule of the design notes, using only the oracle.

Limb rule: q = q0 q1 with q0, q1 primes = 1 mod 2n (so both rings split and
the negacyclic transforms exist); q0 the largest such prime below
2^ceil(b/2), q1 one below 2^floor(b/2), b = ceil(lg q) of Table 2, chosen
among those with 2^(b-1) < q0 q1 < 2^b so that |q mod t| (centred) is
smallest: that residue multiplies the wrap term of the plaintext product in
the decryption noise, so a small one keeps the noise of SIMDScMult low.

Usage: python -m oracle.bfv_params
"""
from __future__ import annotations

import os

from oracle.bfv import BfvOracle

# (name, p_E, ceil(lg q)) of Table 2, n = 2048
TABLE2 = [("binary", 12289, 45), ("medium", 147457, 53), ("high", 2363393, 60)]
N = 2048
OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden", "bfv_params.txt")


def limbs(orc: BfvOracle, t: int, bits: int, n: int = N):
    b0, b1 = (bits + 1) // 2, bits // 2
    step = 2 * n
    q0 = ((1 << b0) - 1) // step * step + 1
    while not orc.is_prime(q0):
        q0 -= step
    best = None
    q1 = ((1 << b1) - 1) // step * step + 1
    while q1 > (1 << (b1 - 1)):
        if q1 != q0 and orc.is_prime(q1) and (1 << (bits - 1)) < q0 * q1 < (1 << bits):
            r = (q0 * q1) % t
            rc = min(r, t - r)
            if best is None or rc < best[0]:
                best = (rc, q1)
        q1 -= step
    return q0, best[1]


def main():
    orc = BfvOracle()
    lines = ["# Packed (BFV/RLWE) parameter sets: name t q0 q1 n",
             "# t = p_E and ceil(lg q) from Table 2 (ENSEI-NTT), n = 2048; q = q0 q1 by the limb rule of",
             "# oracle/bfv_params.py (written by it)"]
    for name, t, bits in TABLE2:
        q0, q1 = limbs(orc, t, bits)
        lines.append(f"{name} {t} {q0} {q1} {N}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
