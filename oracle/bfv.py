"""CPU oracle for the packed (BFV / RLWE) instantiation: ctypes wrapper of
``ensei_bfv_oracle.c``.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it; it shares no code with the GPU library.

Arrays are numpy; residues mod q_l are uint32, a ciphertext is [L=2][2][n]
(limb, word 0 = a^ / word 1 = b^, slot) in evaluation form. The conventions
are written out in the C file's header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ensei_bfv_oracle.c")
LIB = os.path.join(_HERE, "libensei_bfv_oracle.so")
PARAMS = os.path.join(os.path.dirname(_HERE), "tests", "golden", "bfv_params.txt")

u64, i64, i32, vp = C.c_uint64, C.c_int64, C.c_int, C.c_void_p
L = 2  # limbs of q

_SIG = {
    "bo_is_prime": (C.c_int, [u64]),
    "bo_psi": (u64, [u64, i32]),
    "bo_splitmix64": (u64, [u64, u64]),
    "bo_negacyclic": (None, [u64, i32, i64, vp, vp, C.c_int]),
    "bo_delta_mod": (u64, [u64, u64, u64, i32]),
    "bo_encode": (None, [u64, u64, u64, i32, i64, vp, C.c_int, vp]),
    "bo_key": (None, [u64, u64, i32, vp, vp]),
    "bo_encrypt": (None, [u64, u64, u64, i32, i64, vp, vp, vp, u64, u64, vp]),
    "bo_phase": (None, [u64, u64, i32, i64, vp, vp, vp]),
    "bo_decrypt": (None, [u64, u64, u64, i32, i64, vp, vp, vp]),
    "bo_pack": (None, [i64, i32, i64, i32, vp, vp]),
    "bo_filters": (None, [u64, u64, u64, i32, i32, i64, i32, vp, vp]),
    "bo_homconv": (None, [u64, u64, i64, i32, i32, i32, i32, vp, vp, vp, vp]),
    "bo_fold": (None, [u64, i64, i32, i64, i32, vp, vp]),
    "bo_rerand_draws": (None, [u64, u64, i32, i64, C.c_uint32, vp]),
    "bo_rerandomize": (None, [u64, u64, i32, i64, vp, vp, u64, u64, C.c_uint32]),
    "bo_set_threads": (C.c_int, [C.c_int]),
}


def build(src: str = SRC, out: str = LIB, verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra", src, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Params:
    """One parameter set: plaintext modulus t, limbs q0, q1, ring degree n."""

    def __init__(self, name: str, t: int, q0: int, q1: int, n: int):
        self.name, self.t, self.q0, self.q1, self.n = name, t, q0, q1, n

    @property
    def q(self) -> int:
        return self.q0 * self.q1

    @property
    def delta(self) -> int:
        return (self.q + self.t // 2) // self.t

    def __repr__(self):
        return f"Params({self.name}, t={self.t}, q={self.q0}*{self.q1}, n={self.n})"


def table2_params() -> dict:
    """The three parameter sets of Table 2 (Binary, Medium, High), limbs as
    written by oracle/bfv_params.py into tests/golden/bfv_params.txt."""
    out = {}
    for line in open(PARAMS):
        line = line.split("#", 1)[0].split()
        if len(line) == 5:
            name, t, q0, q1, n = line
            out[name] = Params(name, int(t), int(q0), int(q1), int(n))
    return out


def shape_counts(C_: int, F: int, n: int):
    """(P, K, G): channels per slot vector, vectors per channel, vectors per
    image side (the packing of bo_pack)."""
    P = n // F if F <= n else 1
    K = 1 if F <= n else F // n
    return P, K, (C_ + P - 1) // P


class BfvOracle:
    def __init__(self, lib_path: str = LIB):
        if lib_path == LIB and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        self.lib = C.CDLL(lib_path)
        for name, (res, args) in _SIG.items():
            fn = getattr(self.lib, name)
            fn.restype = res
            fn.argtypes = args

    def set_threads(self, k: int) -> int:
        return int(self.lib.bo_set_threads(k))

    def is_prime(self, m: int) -> bool:
        return bool(self.lib.bo_is_prime(m))

    def psi(self, m: int, n: int) -> int:
        return int(self.lib.bo_psi(m, n))

    def splitmix64(self, seed: int, k: int) -> int:
        return int(self.lib.bo_splitmix64(seed % 2**64, k % 2**64))

    def negacyclic(self, x, m: int, inverse: bool = False) -> np.ndarray:
        """x[..., n] (residues < m) -> its negacyclic transform (or inverse) mod m."""
        x = _c(x, np.uint32)
        n = x.shape[-1]
        out = np.empty_like(x)
        self.lib.bo_negacyclic(m, n, x.size // n, _p(x), _p(out), int(inverse))
        return out

    def encode(self, pr: Params, v, scaled: bool) -> np.ndarray:
        """Slot vectors v[..., n] -> evaluation form [..., L, n] (scaled: Delta u; else centred u)."""
        v = _c(v, np.uint32)
        out = np.empty(v.shape[:-1] + (L, pr.n), dtype=np.uint32)
        self.lib.bo_encode(pr.t, pr.q0, pr.q1, pr.n, v.size // pr.n, _p(v), int(scaled), _p(out))
        return out

    def key(self, pr: Params, s) -> np.ndarray:
        s = _c(s, np.int8)
        out = np.empty((L, pr.n), dtype=np.uint32)
        self.lib.bo_key(pr.q0, pr.q1, pr.n, _p(s), _p(out))
        return out

    def encrypt(self, pr: Params, v, s, e, seed_a: int, ct_index0: int = 0) -> np.ndarray:
        """Slot vectors v[..., n], errors e of the same shape -> ct[..., L, 2, n]."""
        v, s, e = _c(v, np.uint32), _c(s, np.int8), _c(e, np.int32)
        assert e.shape == v.shape and s.shape == (pr.n,)
        ct = np.empty(v.shape[:-1] + (L, 2, pr.n), dtype=np.uint32)
        self.lib.bo_encrypt(pr.t, pr.q0, pr.q1, pr.n, v.size // pr.n, _p(v), _p(s), _p(e), seed_a % 2**64,
                            ct_index0 % 2**64, _p(ct))
        return ct

    def phase(self, pr: Params, ct, s) -> np.ndarray:
        """ct[..., L, 2, n] -> phi[..., n] in [0, q) (uint64)."""
        ct, s = _c(ct, np.uint32), _c(s, np.int8)
        count = ct.size // (L * 2 * pr.n)
        phi = np.empty(ct.shape[:-3] + (pr.n,), dtype=np.uint64)
        self.lib.bo_phase(pr.q0, pr.q1, pr.n, count, _p(ct), _p(s), _p(phi))
        return phi

    def decrypt(self, pr: Params, ct, s) -> np.ndarray:
        ct, s = _c(ct, np.uint32), _c(s, np.int8)
        count = ct.size // (L * 2 * pr.n)
        v = np.empty(ct.shape[:-3] + (pr.n,), dtype=np.uint32)
        self.lib.bo_decrypt(pr.t, pr.q0, pr.q1, pr.n, count, _p(ct), _p(s), _p(v))
        return v

    def pack(self, x_hat, n: int) -> np.ndarray:
        """x_hat[B][C][F] -> slot vectors [B][G*K][n]."""
        x_hat = _c(x_hat, np.uint32)
        B, C_, F = x_hat.shape
        P, K, G = shape_counts(C_, F, n)
        v = np.empty((B, G * K, n), dtype=np.uint32)
        self.lib.bo_pack(B, C_, F, n, _p(x_hat), _p(v))
        return v

    def filters(self, pr: Params, w_hat) -> np.ndarray:
        """W^[Cout][Cin][F] -> w_enc[Cout][G][K][L][n]."""
        w_hat = _c(w_hat, np.uint32)
        Cout, Cin, F = w_hat.shape
        P, K, G = shape_counts(Cin, F, pr.n)
        out = np.empty((Cout, G, K, L, pr.n), dtype=np.uint32)
        self.lib.bo_filters(pr.t, pr.q0, pr.q1, Cout, Cin, F, pr.n, _p(w_hat), _p(out))
        return out

    def homconv(self, pr: Params, ct_in, w_enc, mask_enc) -> np.ndarray:
        """ct_in[B][G*K][L][2][n], w_enc[Cout][G][K][L][n], mask_enc[B][Cout*K][L][n] -> ct_out[B][Cout*K][L][2][n]."""
        ct_in, w_enc, mask_enc = _c(ct_in, np.uint32), _c(w_enc, np.uint32), _c(mask_enc, np.uint32)
        Cout, G, K = w_enc.shape[:3]
        B = ct_in.shape[0]
        assert ct_in.shape == (B, G * K, L, 2, pr.n) and mask_enc.shape == (B, Cout * K, L, pr.n)
        out = np.empty((B, Cout * K, L, 2, pr.n), dtype=np.uint32)
        self.lib.bo_homconv(pr.q0, pr.q1, B, G, Cout, K, pr.n, _p(ct_in), _p(w_enc), _p(mask_enc), _p(out))
        return out

    def fold(self, pr: Params, v, F: int) -> np.ndarray:
        """Decrypted output slots v[B][Cout*K][n] -> spectra y[B][Cout][F]."""
        v = _c(v, np.uint32)
        B = v.shape[0]
        P, K, _ = shape_counts(1, F, pr.n)
        Cout = v.shape[1] // K
        y = np.empty((B, Cout, F), dtype=np.uint32)
        self.lib.bo_fold(pr.t, B, Cout, F, pr.n, _p(v), _p(y))
        return y

    def rerand_draws(self, pr: Params, count: int, seed_r: int, flood: int, ct_index0: int = 0) -> np.ndarray:
        """The server's draws for re-randomising `count` ciphertexts: int32 [count][3][n] (rho, e1, e2)."""
        out = np.empty((count, 3, pr.n), dtype=np.int32)
        self.lib.bo_rerand_draws(seed_r % 2**64, ct_index0 % 2**64, pr.n, count, flood, _p(out))
        return out

    def rerandomize(self, pr: Params, ct, pk, seed_r: int, flood: int, ct_index0: int = 0) -> np.ndarray:
        """ct[..., L, 2, n] plus a fresh public-key encryption of zero each (a new array)."""
        ct = np.array(ct, dtype=np.uint32, copy=True, order="C")
        pk = _c(pk, np.uint32)
        assert pk.shape == (L, 2, pr.n)
        count = ct.size // (L * 2 * pr.n)
        self.lib.bo_rerandomize(pr.q0, pr.q1, pr.n, count, _p(ct), _p(pk), seed_r % 2**64, ct_index0 % 2**64, flood)
        return ct

    def secure_conv(self, pr: Params, x_hat, w_hat, r, s, e, seed_a: int):
        """The packed start round of Fig. 2 on spectra: x_hat[B][Cin][F],
        W^[Cout][Cin][F], masks r[B][Cout*K][n] (slot vectors), errors
        e[B][G*K][n]. Returns every intermediate; 'y' (the client's folded
        spectra) equals sum_i W^ x^ + fold(r) mod t."""
        B, Cin, F = x_hat.shape
        v_in = self.pack(x_hat, pr.n)
        ct_in = self.encrypt(pr, v_in, s, e, seed_a)
        w_enc = self.filters(pr, w_hat)
        mask_enc = self.encode(pr, r, scaled=True)
        ct_out = self.homconv(pr, ct_in, w_enc, mask_enc)
        v_out = self.decrypt(pr, ct_out, s)
        y = self.fold(pr, v_out, F)
        return dict(v_in=v_in, ct_in=ct_in, w_enc=w_enc, mask_enc=mask_enc, ct_out=ct_out, v_out=v_out, y=y,
                    r_fold=self.fold(pr, r, F))


_default = None


def default() -> BfvOracle:
    global _default
    if _default is None:
        _default = BfvOracle()
    return _default
