"""Thin Python binding of the packed (BFV / RLWE) calls of libensei.so
(include/ensei_bfv.h): argument marshalling only, every step runs in the HIP
kernels; without the library or a GPU every call raises.

Layouts (uint32 unless stated): spectra [B][C][F]; key s_hat [2][2][n];
ciphertexts [count][2 limbs][2 words][n]; filters [Cout][G][K][2][2][n];
masks as slot vectors [count][n] and encoded [count][2][n]; decrypted slot
vectors [count][n].
"""
from __future__ import annotations

import ctypes as C

import torch

from .ensei import _check, _ptr, lib

_vp, _i32, _i64, _u32, _u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64

SIGNATURES = {
    "ensei_bfv_ctx_create": (_i32, [C.POINTER(_vp), _u32, _u32, _u32, _i32, _i32]),
    "ensei_bfv_ctx_destroy": (_i32, [_vp]),
    "ensei_bfv_key": (_i32, [_vp, _vp, _vp, _vp]),
    "ensei_bfv_encrypt": (_i32, [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _u64, _u64, _vp, _vp]),
    "ensei_bfv_encode_filters": (_i32, [_vp, _vp, _i32, _i32, _i64, _vp, _vp]),
    "ensei_bfv_encode_masks": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "ensei_bfv_homconv": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i64, _vp, _vp]),
    "ensei_bfv_decrypt": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "ensei_bfv_fold": (_i32, [_vp, _vp, _i64, _i32, _i64, _i32, _vp, _vp]),
    "ensei_bfv_rerandomize": (_i32, [_vp, _vp, _i64, _vp, _u64, _u64, _u32, _vp]),
    "ensei_bfv_vectors": (_i64, [_vp, _i32, _i64]),
}

_bound = False


def _lib():
    global _bound
    l = lib()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return l


def geometry(C_: int, F: int, n: int):
    """(P, K, G): channels per slot vector, vectors per channel, vectors per chunk."""
    P = n // F if F <= n else 1
    K = 1 if F <= n else F // n
    return P, K, (C_ + P - 1) // P


class BfvContext:
    """A packed-instantiation context (ensei_bfv_ctx) for (t, q0, q1, n) on one GPU."""

    def __init__(self, t: int, q0: int, q1: int, n: int, device: int | None = None):
        self.device = torch.cuda.current_device() if device is None else device
        self.t, self.q0, self.q1, self.n = t, q0, q1, n
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib().ensei_bfv_ctx_create(C.byref(h), t, q0, q1, n, self.device), "ensei_bfv_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            _lib().ensei_bfv_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _call(self, name, *args):
        with torch.cuda.device(self.device):
            _check(getattr(_lib(), name)(self._h, *args, self._stream()), name)

    def _dev(self, t, name, dtype, numel=None):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must be a tensor on cuda:{self.device}")
        if t.dtype != dtype or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {dtype} tensor")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name} holds {t.numel()} elements, {numel} expected")
        return t

    def _empty(self, shape, dtype=torch.uint32):
        return torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")

    def vectors(self, C_: int, F: int) -> int:
        return int(_lib().ensei_bfv_vectors(self._h, C_, F))

    def key(self, s, out=None):
        self._dev(s, "s", torch.int8, self.n)
        out = self._empty((2, 2, self.n)) if out is None else self._dev(out, "out", torch.uint32, 4 * self.n)
        self._call("ensei_bfv_key", _ptr(s), _ptr(out))
        return out

    def encrypt(self, x_hat, s_hat, e, seed_a: int, ct_index0: int = 0, out=None):
        """x_hat [B][C][F], e [B*G*K][n] -> ct [B*G*K][2][2][n]."""
        self._dev(x_hat, "x_hat", torch.uint32)
        B, C_, F = x_hat.shape
        nv = B * self.vectors(C_, F)
        self._dev(s_hat, "s_hat", torch.uint32, 4 * self.n)
        self._dev(e, "e", torch.int32, nv * self.n)
        out = self._empty((nv, 2, 2, self.n)) if out is None else self._dev(out, "out", torch.uint32, nv * 4 * self.n)
        self._call("ensei_bfv_encrypt", _ptr(x_hat), B, C_, F, _ptr(s_hat), _ptr(e), seed_a % 2**64,
                   ct_index0 % 2**64, _ptr(out))
        return out

    def encode_filters(self, w_hat, out=None):
        """W^ [Cout][Cin][F] -> w_enc [Cout][G][K][2][2][n]."""
        self._dev(w_hat, "w_hat", torch.uint32)
        Cout, Cin, F = w_hat.shape
        P, K, G = geometry(Cin, F, self.n)
        shape = (Cout, G, K, 2, 2, self.n)
        out = self._empty(shape) if out is None else self._dev(out, "out", torch.uint32, Cout * G * K * 4 * self.n)
        self._call("ensei_bfv_encode_filters", _ptr(w_hat), Cout, Cin, F, _ptr(out))
        return out

    def encode_masks(self, r, out=None):
        """r [..., n] slot vectors -> [..., 2, n]."""
        self._dev(r, "r", torch.uint32)
        count = r.numel() // self.n
        out = self._empty(tuple(r.shape[:-1]) + (2, self.n)) if out is None else self._dev(
            out, "out", torch.uint32, count * 2 * self.n)
        self._call("ensei_bfv_encode_masks", _ptr(r), count, _ptr(out))
        return out

    def homconv(self, ct_in, w_enc, mask_enc, B: int, Cin: int, F: int, out=None):
        """ct_in [B*G*K][2][2][n], w_enc [Cout][G][K][2][2][n], mask_enc [B*Cout*K][2][n] -> [B*Cout*K][2][2][n]."""
        Cout = w_enc.shape[0]
        P, K, G = geometry(Cin, F, self.n)
        self._dev(ct_in, "ct_in", torch.uint32, B * G * K * 4 * self.n)
        self._dev(w_enc, "w_enc", torch.uint32, Cout * G * K * 4 * self.n)
        self._dev(mask_enc, "mask_enc", torch.uint32, B * Cout * K * 2 * self.n)
        nout = B * Cout * K
        out = self._empty((nout, 2, 2, self.n)) if out is None else self._dev(out, "out", torch.uint32, nout * 4 * self.n)
        self._call("ensei_bfv_homconv", _ptr(ct_in), _ptr(w_enc), _ptr(mask_enc), B, Cin, Cout, F, _ptr(out))
        return out

    def decrypt(self, ct, s_hat, out=None):
        """ct [count][2][2][n] -> slot vectors [count][n]."""
        self._dev(ct, "ct", torch.uint32)
        count = ct.numel() // (4 * self.n)
        self._dev(s_hat, "s_hat", torch.uint32, 4 * self.n)
        out = self._empty((count, self.n)) if out is None else self._dev(out, "out", torch.uint32, count * self.n)
        self._call("ensei_bfv_decrypt", _ptr(ct), _ptr(s_hat), count, _ptr(out))
        return out

    def rerandomize(self, ct, pk, seed_r: int, flood: int, ct_index0: int = 0):
        """In place: each ciphertext of ct [count][2][2][n] gains a fresh
        public-key encryption of zero under pk [2][2][n] (circuit privacy)."""
        self._dev(ct, "ct", torch.uint32)
        self._dev(pk, "pk", torch.uint32, 4 * self.n)
        self._call("ensei_bfv_rerandomize", _ptr(ct), ct.numel() // (4 * self.n), _ptr(pk), seed_r % 2**64,
                   ct_index0 % 2**64, int(flood))
        return ct

    def fold(self, v, B: int, C_: int, F: int, negate: bool = False, out=None):
        """Slot vectors v [B*C*K][n] -> spectra [B][C][F] (negate: -y mod t)."""
        P, K, _ = geometry(1, F, self.n)
        self._dev(v, "v", torch.uint32, B * C_ * K * self.n)
        out = self._empty((B, C_, F)) if out is None else self._dev(out, "out", torch.uint32, B * C_ * F)
        self._call("ensei_bfv_fold", _ptr(v), B, C_, F, int(negate), _ptr(out))
        return out
