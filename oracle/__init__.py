"""CPU oracle for the ENSEI secure-convolution hot path: ctypes wrapper.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library (``paper_2003_05328_amd``) and never imports it; the
product path fails loudly rather than falling back here.

Every function takes and returns numpy arrays and follows the plain
definitions written out in ``ensei_oracle.c`` (see that file's header for the
conventions and the paper passages they restate).
"""
from __future__ import annotations

import ctypes as C
import importlib
import os
from decimal import ROUND_FLOOR, Decimal, localcontext

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libensei_oracle.so")

u64, i64, i32, vp = C.c_uint64, C.c_int64, C.c_int, C.c_void_p

_SIG = {
    "or_is_prime": (C.c_int, [u64]),
    "or_primitive_root": (u64, [u64]),
    "or_root_of_unity": (u64, [u64, u64, C.c_int]),
    "or_inverse": (u64, [u64, u64]),
    "or_dft2d_direct": (None, [u64, i64, i32, i32, vp, vp, C.c_int]),
    "or_ntt2d": (None, [u64, i64, i32, i32, vp, vp, C.c_int]),
    "or_weight_prep": (None, [u64, i32, i32, i32, i32, i32, i32, vp, vp]),
    "or_cyclic_conv": (None, [u64, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp]),
    "or_splitmix64": (u64, [u64, u64]),
    "or_delta": (u64, [u64]),
    "or_encrypt": (None, [u64, i64, i32, i64, i32, vp, vp, vp, u64, u64, vp]),
    "or_phase": (u64, [i32, vp, i64, vp]),
    "or_decrypt": (None, [u64, i64, i32, i64, i32, vp, vp, vp]),
    "or_expand_seeded": (None, [i64, i32, i64, i32, u64, u64, vp, vp]),
    "or_sample_errors": (None, [vp, i32, u64, u64, i64, i32, i64, vp]),
    "or_homconv": (None, [u64, i32, i32, i32, i64, i32, vp, vp, vp, vp]),
    "or_homconv_select": (None, [u64, i32, i32, i32, i64, i32, vp, vp, vp, i64, vp, vp]),
    "or_server_share": (None, [u64, i64, i32, i32, vp, vp]),
    "or_homrec": (None, [u64, i64, i32, i64, i32, vp, vp]),
    "or_reshare": (None, [u64, i64, vp, vp, vp, C.c_int, vp]),
    "or_set_threads": (C.c_int, [C.c_int]),
}


def _c(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """The oracle functions bound to one build of ``ensei_oracle.c``."""

    def __init__(self, lib_path: str = _LIB_PATH):
        if lib_path == _LIB_PATH and not os.path.exists(lib_path):
            # import the submodule by name: ``from . import build`` would first
            # look the name up through this module's __getattr__
            importlib.import_module(__name__ + ".build").build()
        lib = C.CDLL(lib_path)
        for name, (res, args) in _SIG.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        self.lib = lib
        self.path = lib_path

    def set_threads(self, k: int) -> int:
        """Thread count for the oracle's OpenMP loops; returns the count in effect."""
        return self.lib.or_set_threads(int(k))

    def is_prime(self, p: int) -> bool:
        return bool(self.lib.or_is_prime(p))

    def primitive_root(self, p: int) -> int:
        return int(self.lib.or_primitive_root(p))

    def root_of_unity(self, p: int, N: int, inverse: bool = False) -> int:
        return int(self.lib.or_root_of_unity(p, N, int(inverse)))

    def inverse(self, a: int, p: int) -> int:
        return int(self.lib.or_inverse(a, p))

    def delta(self, p: int) -> int:
        return int(self.lib.or_delta(p))

    def splitmix64(self, seed: int, k: int) -> int:
        return int(self.lib.or_splitmix64(seed % 2**64, k % 2**64))

    def dft2d_direct(self, x: np.ndarray, p: int, inverse: bool = False) -> np.ndarray:
        """O(F^2) double-sum 2D DFT over Z_p of x[..., H, W] (uint32)."""
        x = _c(x, np.uint32)
        H, W = x.shape[-2:]
        out = np.empty_like(x)
        self.lib.or_dft2d_direct(p, x.size // (H * W), H, W, _p(x), _p(out), int(inverse))
        return out

    def ntt2d(self, x: np.ndarray, p: int, inverse: bool = False) -> np.ndarray:
        """2D transform of x[..., H, W] evaluated axis by axis (plain 1D sums)."""
        x = _c(x, np.uint32)
        H, W = x.shape[-2:]
        out = np.empty_like(x)
        self.lib.or_ntt2d(p, x.size // (H * W), H, W, _p(x), _p(out), int(inverse))
        return out

    def weight_prep(self, w: np.ndarray, H: int, W: int, p: int) -> np.ndarray:
        """w[Cout][Cin][kh][kw] int32 -> W^ [Cout][Cin][H*W] uint32."""
        w = _c(w, np.int32)
        Cout, Cin, kh, kw = w.shape
        out = np.empty((Cout, Cin, H * W), dtype=np.uint32)
        self.lib.or_weight_prep(p, Cout, Cin, kh, kw, H, W, _p(w), _p(out))
        return out

    def cyclic_conv(self, x: np.ndarray, w: np.ndarray, p: int) -> np.ndarray:
        """x[B][Cin][H][W] residues, w[Cout][Cin][kh][kw] ints -> y[B][Cout][H][W] mod p."""
        x = _c(x, np.uint32)
        w = _c(w, np.int32)
        B, Cin, H, W = x.shape
        Cout, Cin2, kh, kw = w.shape
        assert Cin == Cin2
        y = np.empty((B, Cout, H, W), dtype=np.uint32)
        self.lib.or_cyclic_conv(p, B, Cin, Cout, H, W, kh, kw, _p(x), _p(w), _p(y))
        return y

    def encrypt(self, m, s, e, seed_a: int, p: int, ct_index0: int = 0) -> np.ndarray:
        """Encrypt plaintexts m[B][C][F] (errors e of the same shape) into the
        word-major ciphertexts ct[B][F][n+1][C] (word j of ciphertext (b, c, f)
        at ct[b][f][j][c]). A 1-D m is a plain list: B = C = 1, F = N, and the
        result is returned as rows [N][n+1]."""
        m = _c(m, np.uint32)
        e = _c(e, np.int32)
        s = _c(s, np.int8)
        n = s.shape[0]
        flat = m.ndim == 1
        B, C, F = (1, 1, m.shape[0]) if flat else m.shape
        assert e.size == m.size
        ct = np.empty((B, F, n + 1, C), dtype=np.uint64)
        self.lib.or_encrypt(p, B, C, F, n, _p(m), _p(s), _p(e), seed_a % 2**64, ct_index0 % 2**64, _p(ct))
        return ct.reshape(F, n + 1) if flat else ct

    def phase(self, ct_row: np.ndarray, s: np.ndarray) -> int:
        """phi = b - <a, s> of one ciphertext given as its n+1 words."""
        row = _c(ct_row, np.uint64)
        s = _c(s, np.int8)
        return int(self.lib.or_phase(s.shape[0], _p(row), 1, _p(s)))

    def decrypt(self, ct: np.ndarray, s: np.ndarray, p: int) -> np.ndarray:
        """ct[B][F][n+1][C] -> m[B][C][F]; a 2-D ct[N][n+1] is a plain list -> m[N]."""
        s = _c(s, np.int8)
        n = s.shape[0]
        ct = _c(ct, np.uint64)
        flat = ct.ndim == 2
        B, F, n1, C = (1, ct.shape[0], ct.shape[1], 1) if flat else ct.shape
        assert n1 == n + 1
        m = np.empty((B, C, F), dtype=np.uint32)
        self.lib.or_decrypt(p, B, C, F, n, _p(ct), _p(s), _p(m))
        return m.reshape(F) if flat else m

    def expand_seeded(self, bw, n: int, seed_a: int, ct_index0: int = 0) -> np.ndarray:
        """Seeded ciphertexts (Sec. 5.1: the public constants generated
        offline): b words bw[B][F][C] -> ct[B][F][n+1][C], word j < n of
        ciphertext (b, c, f) the generator's output (ct_index0 + q) n + j + 1."""
        bw = _c(bw, np.uint64)
        B, F, C = bw.shape
        ct = np.empty((B, F, n + 1, C), dtype=np.uint64)
        self.lib.or_expand_seeded(B, C, F, n, seed_a % 2**64, ct_index0 % 2**64, _p(bw), _p(ct))
        return ct

    def encrypt_seeded(self, m, s, e, seed_a: int, p: int, ct_index0: int = 0) -> np.ndarray:
        """What a client sends for seeded ciphertexts: the b words of Enc,
        bw[B][F][C] = Enc(m)[b][f][n][c] (the a-words follow from seed_a)."""
        n = np.asarray(s).shape[0]
        return np.ascontiguousarray(self.encrypt(m, s, e, seed_a, p, ct_index0)[:, :, n, :])

    def homconv_seeded(self, bw, n: int, seed_a: int, w_hat, r, p: int, ct_index0: int = 0) -> np.ndarray:
        """HomConv of the seeded ciphertexts given by (seed_a, ct_index0, bw)."""
        return self.homconv(self.expand_seeded(bw, n, seed_a, ct_index0), w_hat, r, p)

    def sample_errors(self, seed_e: int, B: int, C: int, F: int, ct_index0: int = 0) -> np.ndarray:
        """Errors e[B][C][F] of the rounded Gaussian (sigma 3.2) drawn from the
        public generator seeded with seed_e (or_sample_errors, thresholds from
        cdt_table)."""
        T = np.array(cdt_table(), dtype=np.uint64)
        e = np.empty((B, C, F), dtype=np.int32)
        self.lib.or_sample_errors(_p(T), T.size, seed_e % 2**64, ct_index0 % 2**64, B, C, F, _p(e))
        return e

    def homconv(self, ct_in, w_hat, r, p: int) -> np.ndarray:
        """ct_in[B][F][n+1][Cin], w_hat[Cout][Cin][F], r[B][Cout][F] -> ct_out[B][F][n+1][Cout]."""
        ct_in = _c(ct_in, np.uint64)
        w_hat = _c(w_hat, np.uint32)
        r = _c(r, np.uint32)
        B, F, n1, Cin = ct_in.shape
        Cout = w_hat.shape[0]
        assert w_hat.shape == (Cout, Cin, F) and r.shape == (B, Cout, F)
        out = np.empty((B, F, n1, Cout), dtype=np.uint64)
        self.lib.or_homconv(p, B, Cin, Cout, F, n1 - 1, _p(ct_in), _p(w_hat), _p(r), _p(out))
        return out

    def homconv_select(self, ct_in, w_hat, r, sel, p: int) -> np.ndarray:
        """Output ciphertexts for the (b, o, f) triples in sel[k] -> words [k][n+1]."""
        ct_in = _c(ct_in, np.uint64)
        w_hat = _c(w_hat, np.uint32)
        r = _c(r, np.uint32)
        sel = _c(sel, np.int64).reshape(-1, 3)
        B, F, n1, Cin = ct_in.shape
        Cout = w_hat.shape[0]
        out = np.empty((sel.shape[0], n1), dtype=np.uint64)
        self.lib.or_homconv_select(p, B, Cin, Cout, F, n1 - 1, _p(ct_in), _p(w_hat), _p(r), sel.shape[0], _p(sel), _p(out))
        return out

    def server_share(self, r, H: int, W: int, p: int) -> np.ndarray:
        """r[..., F] -> s_B[..., H, W] = INTT2D(-r mod p)."""
        r = _c(r, np.uint32)
        batch = r.size // (H * W)
        out = np.empty(r.shape[:-1] + (H, W), dtype=np.uint32)
        self.lib.or_server_share(p, batch, H, W, _p(r), _p(out))
        return out

    def homrec(self, ct, s_hat, p: int) -> np.ndarray:
        """HomRec: ct[B][F][n+1][C] with Delta * s_hat[B][C][F] added to every b word (a new array)."""
        ct = np.array(ct, dtype=np.uint64, copy=True, order="C")
        s_hat = _c(s_hat, np.uint32)
        B, F, n1, Cc = ct.shape
        assert s_hat.shape == (B, Cc, F)
        self.lib.or_homrec(p, B, Cc, F, n1 - 1, _p(ct), _p(s_hat))
        return ct

    def reshare(self, s_a, s_b, s_b_next, act: int, p: int) -> np.ndarray:
        """The activation stand-in: s_a' = f(s_a + s_b) - s_b' mod p (act 0 identity, 1 square)."""
        s_a, s_b, s_b_next = _c(s_a, np.uint32), _c(s_b, np.uint32), _c(s_b_next, np.uint32)
        assert s_a.shape == s_b.shape == s_b_next.shape
        out = np.empty_like(s_a)
        self.lib.or_reshare(p, s_a.size, _p(s_a), _p(s_b), _p(s_b_next), act, _p(out))
        return out

    def fdsc_round1(self, r0: dict, inp1, s_b1, act: int, p: int):
        """The next round of Fig. 2 (activation, re-encryption, HomRec, convolution) after round r0 (fdsc_round0's
        result), with the activation replaced by reshare in the clear.

        inp1 holds the next layer (its filters w over Cin = the previous Cout,
        the client's key s, errors e, masks r, seed_a); s_b1 is the server's
        fresh share [B][Cin][H][W]. Returns the round's intermediates: s_a1
        (client's share after the activation), ct_a (Enc of its transform),
        ct_rec (after HomRec), ct_out, m, s_a and s_b (the round's shares).
        """
        S = inp1.shape
        s_a1 = self.reshare(r0["s_a"], r0["s_b"], s_b1, act, p)
        ct_a = self.encrypt(self.ntt2d(s_a1, p).reshape(S.B, S.Cin, S.F), inp1.s, inp1.e, inp1.seed_a, p)
        ct_rec = self.homrec(ct_a, self.ntt2d(s_b1, p).reshape(S.B, S.Cin, S.F), p)
        w_hat = self.weight_prep(inp1.w, S.H, S.W, p)
        ct_out = self.homconv(ct_rec, w_hat, inp1.r, p)
        m = self.decrypt(ct_out, inp1.s, p)
        s_a = self.ntt2d(m.reshape(S.B, S.Cout, S.H, S.W), p, inverse=True)
        s_b = self.server_share(inp1.r, S.H, S.W, p)
        return dict(s_a1=s_a1, ct_a=ct_a, ct_rec=ct_rec, w_hat=w_hat, ct_out=ct_out, m=m, s_a=s_a, s_b=s_b)

    def fdsc_round0(self, inp, p: int):
        """The whole secure convolution of one layer (Fig. 2, round 0) on the CPU.

        Returns a dict with every intermediate: x_hat, w_hat, ct_in, ct_out, m,
        s_a (the client's spatial share) and s_b (the server's spatial share).
        """
        S = inp.shape
        x_hat = self.ntt2d(inp.x, p).reshape(S.B, S.Cin, S.F)
        w_hat = self.weight_prep(inp.w, S.H, S.W, p)
        ct_in = self.encrypt(x_hat, inp.s, inp.e, inp.seed_a, p)  # [B][F][n+1][Cin]
        ct_out = self.homconv(ct_in, w_hat, inp.r, p)  # [B][F][n+1][Cout]
        m = self.decrypt(ct_out, inp.s, p)  # [B][Cout][F]
        s_a = self.ntt2d(m.reshape(S.B, S.Cout, S.H, S.W), p, inverse=True)
        s_b = self.server_share(inp.r, S.H, S.W, p)
        return dict(x_hat=x_hat, w_hat=w_hat, ct_in=ct_in, ct_out=ct_out, m=m, s_a=s_a, s_b=s_b)


_default: Oracle | None = None


CDT_BITS = 48  # grid of the error sampler's thresholds
CDT_SIZE = 32  # thresholds: |e| <= 32
SIGMA_NUM, SIGMA_DEN = 16, 5  # sigma = 3.2


def _pi(prec_digits: int) -> Decimal:
    """pi = 16 arctan(1/5) - 4 arctan(1/239) (Machin), each arctan by its
    alternating series, in decimal arithmetic of the current precision."""
    def arctan_inv(m: int) -> Decimal:
        total, term, k, sign = Decimal(0), Decimal(1) / m, 1, 1
        m2 = m * m
        while term > Decimal(10) ** (-prec_digits - 5):
            total += sign * term / k
            term /= m2
            k += 2
            sign = -sign
        return total

    return 16 * arctan_inv(5) - 4 * arctan_inv(239)


def _erf(x: Decimal, prec_digits: int) -> Decimal:
    """erf(x) = 2/sqrt(pi) exp(-x^2) sum_n 2^n x^(2n+1) / (2n+1)!! (all terms
    positive), summed until the terms fall below the working precision."""
    term, total, n = x, Decimal(0), 0
    x2 = x * x
    while term > Decimal(10) ** (-prec_digits - 5) * (total + 1):
        total += term
        n += 1
        term = term * 2 * x2 / (2 * n + 1)
    return 2 / _pi(prec_digits).sqrt() * (-x2).exp() * total


def cdt_table() -> list:
    """T[k] = floor(2^48 P(|e| <= k)) for e the rounded N(0, sigma^2), i.e.
    floor(2^48 erf((k + 1/2) / (sigma sqrt 2))), k < 32, in 80-digit decimal
    arithmetic (far below the 2^-48 grid)."""
    prec = 80
    with localcontext() as ctx:
        ctx.prec = prec
        sigma = Decimal(SIGMA_NUM) / SIGMA_DEN
        out = []
        for k in range(CDT_SIZE):
            x = (Decimal(k) + Decimal(1) / 2) / (sigma * Decimal(2).sqrt())
            v = (Decimal(2) ** CDT_BITS * _erf(x, prec)).to_integral_value(rounding=ROUND_FLOOR)
            out.append(min(int(v), 2**CDT_BITS - 1))
        return out


def default() -> Oracle:
    """The oracle built from the committed source (built on first use)."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def __getattr__(name):
    # module-level access (oracle.ntt2d, ...) forwards to the default build
    if name.startswith("_"):
        raise AttributeError(name)
    return getattr(default(), name)
