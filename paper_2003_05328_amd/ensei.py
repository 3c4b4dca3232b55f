"""Thin Python binding of libensei.so (argument marshalling only).

Every operation runs in the HIP kernels behind the C ABI declared in
``include/ensei.h``; this module only checks tensor dtypes, shapes and
devices, passes ``data_ptr()`` values and the current HIP stream, and turns
status codes into exceptions. PyTorch provides device memory and streams.
There is no CPU path: without the built library or a GPU every call raises.

Names follow the C ABI: ``ensei_ntt2d`` -> ``Context.ntt2d`` and so on; the
raw ctypes functions are available as ``lib().ensei_ntt2d`` etc.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libensei.so")
# the vector-ALU comparison kernel (include/ensei_bench.h), outside the product library
BENCH_LIB_PATH = os.path.join(_HERE, "libensei_bench.so")

ENSEI_OK = 0
STATUS = {
    -1: "ENSEI_ERR_ARG",
    -2: "ENSEI_ERR_SHAPE",
    -3: "ENSEI_ERR_MODULUS",
    -4: "ENSEI_ERR_ALIGN",
    -5: "ENSEI_ERR_OVERLAP",
    -6: "ENSEI_ERR_LIMIT",
    -7: "ENSEI_ERR_DEVICE",
    -8: "ENSEI_ERR_HIP",
    -9: "ENSEI_ERR_TIMEOUT",
    -10: "ENSEI_ERR_BUDGET",
    -11: "ENSEI_ERR_CANCELLED",
    -12: "ENSEI_ERR_STATE",
}

_vp, _i32, _i64, _u32, _u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64

# name -> (restype, argtypes); the same table drives the symbol-export test.
SIGNATURES = {
    "ensei_ctx_create": (_i32, [C.POINTER(_vp), _u32, _i32]),
    "ensei_ctx_destroy": (_i32, [_vp]),
    "ensei_status_str": (C.c_char_p, [_i32]),
    "ensei_ctx_device": (_i32, [_vp]),
    "ensei_ctx_modulus": (_u32, [_vp]),
    "ensei_ctx_delta": (_u64, [_vp]),
    "ensei_ctx_max_dim": (_i32, [_vp]),
    "ensei_ntt2d": (_i32, [_vp, _vp, _vp, _i64, _i32, _i32, _vp]),
    "ensei_intt2d": (_i32, [_vp, _vp, _vp, _i64, _i32, _i32, _vp]),
    "ensei_server_share": (_i32, [_vp, _vp, _vp, _i64, _i32, _i32, _vp]),
    "ensei_weight_prep": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp]),
    "ensei_wpack_bytes": (C.c_size_t, [_i32, _i32, _i64]),
    "ensei_pack_weights": (_i32, [_vp, _vp, _i32, _i32, _i64, _vp, _vp]),
    "ensei_encrypt": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i64, _i32, _u64, _u64, _vp, _vp]),
    "ensei_homconv": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i64, _i32, _vp, _vp]),
    "ensei_sample_errors": (_i32, [_vp, _u64, _u64, _i64, _i32, _i64, _vp, _vp]),
    "ensei_error_table": (_i32, [_vp, _vp, _i32]),
    "ensei_encrypt_seeded": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i64, _i32, _u64, _u64, _vp, _vp]),
    "ensei_homconv_seeded": (_i32, [_vp, _vp, _u64, _u64, _vp, _vp, _i64, _i32, _i32, _i64, _i32, _vp, _vp]),
    "ensei_decrypt": (_i32, [_vp, _vp, _vp, _i64, _i32, _i64, _i32, _vp, _vp]),
    "ensei_homrec": (_i32, [_vp, _vp, _vp, _i64, _i32, _i64, _i32, _vp]),
    "ensei_homrec_seeded": (_i32, [_vp, _vp, _vp, _i64, _i32, _i64, _vp]),
    "ensei_reshare": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp]),
    "ensei_plan_create": (_i32, [_vp, _vp, _i32, C.c_char_p, C.POINTER(_vp)]),
    "ensei_plan_create_seeded": (_i32, [_vp, _vp, _i32, C.c_char_p, C.POINTER(_vp)]),
    "ensei_plan_run": (_i32, [_vp, _vp]),
    "ensei_plan_run_stage": (_i32, [_vp, _i32, _vp]),
    "ensei_plan_schedule": (_i32, [_vp, _vp]),
    "ensei_plan_destroy": (_i32, [_vp]),
    "ensei_request_bytes": (C.c_size_t, [_vp]),
    "ensei_server_create": (_i32, [_vp, C.c_size_t, _i32, _i32, C.POINTER(_vp)]),
    "ensei_server_create_seeded": (_i32, [_vp, C.c_size_t, _i32, _i32, C.POINTER(_vp)]),
    "ensei_server_add_shape": (_i32, [_vp, _vp, _vp, C.POINTER(_i32)]),
    "ensei_server_submit": (_i32, [_vp, _i32, _vp, C.POINTER(_u64)]),
    "ensei_server_cancel": (_i32, [_vp, _u64]),
    "ensei_server_set_queue_limit": (_i32, [_vp, C.c_size_t]),
    "ensei_server_clock": (_i32, [_vp, C.POINTER(C.c_double)]),
    "ensei_server_poll": (_i32, [_vp, _u64, _vp]),
    "ensei_server_wait": (_i32, [_vp, _u64, _i32]),
    "ensei_server_forget": (_i32, [_vp, _u64]),
    "ensei_server_stats": (_i32, [_vp, _vp]),
    "ensei_server_destroy": (_i32, [_vp]),
}


BENCH_SIGNATURES = {
    "ensei_bench_homconv_valu": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i64, _i32, _vp, _vp]),
}


class ShapeDesc(C.Structure):
    """``ensei_shape``: the shape of one secure convolution."""

    _fields_ = [(f, _i32) for f in ("H", "W", "Cin", "Cout", "kh", "kw", "n")]


class RequestDesc(C.Structure):
    """``ensei_request``: one request's device buffers."""

    _fields_ = [("x", _vp), ("s", _vp), ("e", _vp), ("r", _vp), ("seed_a", _u64), ("s_a", _vp), ("s_b", _vp),
                ("stream", _vp)]


class RequestInfo(C.Structure):
    """``ensei_request_info``."""

    _fields_ = [("state", _i32), ("status", _i32), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]


class ServerInfo(C.Structure):
    """``ensei_server_info``."""

    _fields_ = [(f, _u64) for f in ("budget_bytes", "used_bytes", "peak_used_bytes", "queued", "inflight_batches",
                                    "completed", "failed", "batches", "cancelled", "refused")]


class LayerDesc(C.Structure):
    """``ensei_layer``: one layer of a batched plan."""

    _fields_ = [(f, _i32) for f in ("H", "W", "Cin", "Cout", "kh", "kw", "n")] + [
        ("batch", _i64),
        ("seed_a", _u64),
    ] + [(f, _vp) for f in ("w", "x", "s", "e", "r", "x_hat", "ct_in", "ct_out", "m", "s_a", "s_b")]


class ScheduleDesc(C.Structure):
    """``ensei_schedule``: the HomConv tile schedule a plan runs."""

    _fields_ = [("blocks", _i32), ("from_cache", _i32), ("chunk", _i64), ("homconv_us", C.c_double),
                ("shared_layers", _i32), ("own_layers", _i32), ("branches", _i32), ("pad", _i32),
                ("serial_us", C.c_double), ("branches_us", C.c_double)]


class EnseiError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        name = STATUS.get(status, str(status))
        msg = _lib.ensei_status_str(status).decode() if _lib is not None else ""
        super().__init__(f"{where}: {name} ({msg})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2003_05328_amd.build` "
                "(there is no CPU fallback)"
            )
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


_bench_lib = None


def bench_lib():
    """libensei_bench.so (comparison kernels for benchmarks and tests)."""
    global _bench_lib
    if _bench_lib is None:
        lib()
        if not os.path.exists(BENCH_LIB_PATH):
            raise RuntimeError(f"{BENCH_LIB_PATH} is missing: build it with `python -m paper_2003_05328_amd.build`")
        l = C.CDLL(BENCH_LIB_PATH)
        for name, (res, args) in BENCH_SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _bench_lib = l
    return _bench_lib


def _check(status: int, where: str):
    if status != ENSEI_OK:
        raise EnseiError(status, where)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A library context for prime p on one GPU (``ensei_ctx``)."""

    def __init__(self, p: int = 65537, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ENSEI kernels run only on the GPU")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ensei_ctx_create(C.byref(h), p, self.device), "ensei_ctx_create")
        self._h = h
        self.p = int(lib().ensei_ctx_modulus(h))
        self.delta = int(lib().ensei_ctx_delta(h))
        self.max_dim = int(lib().ensei_ctx_max_dim(h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            lib().ensei_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, t: torch.Tensor, name: str, dtype):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must live on cuda:{self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")

    def _out(self, out, shape, dtype):
        """A new output of `shape`, or the caller's, which must hold exactly as
        many elements (the kernels write all of them)."""
        if out is None:
            return self._empty(shape, dtype)
        self._dev(out, "out", dtype)
        need = 1
        for d in shape:
            need *= int(d)
        if out.numel() != need:
            raise ValueError(f"out holds {out.numel()} elements, {need} are written")
        return out

    def _call(self, name, *args):
        with torch.cuda.device(self.device):
            _check(getattr(lib(), name)(self._h, *args, self._stream()), name)

    # -- transforms ---------------------------------------------------------
    def ntt2d(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """x uint32 [..., H, W] -> out uint32 [..., H*W] (ensei_ntt2d)."""
        self._dev(x, "x", torch.uint32)
        H, W = x.shape[-2:]
        batch = x.numel() // (H * W)
        out = self._out(out, x.shape[:-2] + (H * W,), torch.uint32)
        self._call("ensei_ntt2d", _ptr(x), _ptr(out), batch, H, W)
        return out

    def intt2d(self, X: torch.Tensor, H: int, W: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """X uint32 [..., H*W] -> out uint32 [..., H, W] (ensei_intt2d)."""
        self._dev(X, "X", torch.uint32)
        batch = X.numel() // (H * W)
        out = self._out(out, X.shape[:-1] + (H, W), torch.uint32)
        self._call("ensei_intt2d", _ptr(X), _ptr(out), batch, H, W)
        return out

    def server_share(self, r: torch.Tensor, H: int, W: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """r uint32 [..., H*W] -> s_B = INTT2D(-r) uint32 [..., H, W] (ensei_server_share)."""
        self._dev(r, "r", torch.uint32)
        batch = r.numel() // (H * W)
        out = self._out(out, r.shape[:-1] + (H, W), torch.uint32)
        self._call("ensei_server_share", _ptr(r), _ptr(out), batch, H, W)
        return out

    # -- weights -------------------------------------------------------------
    def weight_prep(self, w: torch.Tensor, H: int, W: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """w int32 [Cout][Cin][kh][kw] -> W^ uint32 [Cout][Cin][H*W] (ensei_weight_prep)."""
        self._dev(w, "w", torch.int32)
        Cout, Cin, kh, kw = w.shape
        out = self._out(out, (Cout, Cin, H * W), torch.uint32)
        self._call("ensei_weight_prep", _ptr(w), Cout, Cin, kh, kw, H, W, _ptr(out))
        return out

    def pack_weights(self, w_hat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """W^ uint32 [Cout][Cin][F] -> packed int8 limbs (ensei_pack_weights)."""
        self._dev(w_hat, "w_hat", torch.uint32)
        Cout, Cin, F = w_hat.shape
        nb = int(lib().ensei_wpack_bytes(Cout, Cin, F))
        out = self._out(out, (nb,), torch.int8)
        if out.numel() < nb:
            raise ValueError(f"packed-weight buffer needs {nb} bytes")
        self._call("ensei_pack_weights", _ptr(w_hat), Cout, Cin, F, _ptr(out))
        return out

    # -- LWE -----------------------------------------------------------------
    def encrypt(self, m, s, e, seed_a: int, ct_index0: int = 0, out=None) -> torch.Tensor:
        """m uint32 [B][C][F] (or [N]), s int8 [n], e int32 like m -> word-major
        ct uint64 [B][F][n+1][C] (or [N][n+1] for a 1-D list) (ensei_encrypt)."""
        self._dev(m, "m", torch.uint32)
        self._dev(s, "s", torch.int8)
        self._dev(e, "e", torch.int32)
        if e.numel() != m.numel():
            raise ValueError("e must have one error per plaintext")
        n = s.numel()
        flat = m.dim() == 1
        B, C, F = (1, 1, m.shape[0]) if flat else tuple(m.shape)
        shape = (F, n + 1) if flat else (B, F, n + 1, C)
        out = self._out(out, shape, torch.uint64)
        if out.numel() != B * C * F * (n + 1):
            raise ValueError("ct has the wrong size")
        self._call("ensei_encrypt", _ptr(m), _ptr(s), _ptr(e), B, C, F, n, seed_a % 2**64, ct_index0 % 2**64, _ptr(out))
        return out

    def sample_errors(self, seed_e: int, B: int, C: int, F: int, ct_index0: int = 0, out=None) -> torch.Tensor:
        """Errors int32 [B][C][F] of the rounded Gaussian (sigma 3.2) from the
        public generator seeded with seed_e (ensei_sample_errors)."""
        out = self._out(out, (B, C, F), torch.int32)
        self._call("ensei_sample_errors", seed_e % 2**64, ct_index0 % 2**64, B, C, F, _ptr(out))
        return out

    def error_table(self) -> list:
        """The error sampler's 32 thresholds as computed by the library (ensei_error_table)."""
        buf = (C.c_uint64 * 32)()
        n = lib().ensei_error_table(self._h, buf, 32)
        if n != 32:
            raise EnseiError(n, "ensei_error_table")
        return [int(x) for x in buf]

    def encrypt_seeded(self, m, s, e, seed_a: int, ct_index0: int = 0, out=None) -> torch.Tensor:
        """Seeded ciphertexts: m uint32 [B][C][F], s, e as encrypt -> only the
        b words, uint64 [B][F][C] (ensei_encrypt_seeded); the a-words follow
        from (seed_a, ct_index0)."""
        self._dev(m, "m", torch.uint32)
        self._dev(s, "s", torch.int8)
        self._dev(e, "e", torch.int32)
        if m.dim() != 3 or e.numel() != m.numel():
            raise ValueError("m must be [B][C][F] with one error per plaintext")
        B, C, F = tuple(m.shape)
        out = self._out(out, (B, F, C), torch.uint64)
        self._call("ensei_encrypt_seeded", _ptr(m), _ptr(s), _ptr(e), B, C, F, s.numel(), seed_a % 2**64,
                   ct_index0 % 2**64, _ptr(out))
        return out

    def decrypt(self, ct, s, out=None) -> torch.Tensor:
        """Word-major ct uint64 [B][F][n+1][C] (or rows [N][n+1]), s int8 [n] ->
        m uint32 [B][C][F] (or [N]) (ensei_decrypt)."""
        self._dev(ct, "ct", torch.uint64)
        self._dev(s, "s", torch.int8)
        n = s.numel()
        flat = ct.dim() == 2
        if flat:
            B, F, n1, C = 1, ct.shape[0], ct.shape[1], 1
        else:
            B, F, n1, C = tuple(ct.shape)
        if n1 != n + 1:
            raise ValueError("ciphertexts must have n+1 words")
        shape = (F,) if flat else (B, C, F)
        out = self._out(out, shape, torch.uint32)
        self._call("ensei_decrypt", _ptr(ct), _ptr(s), B, C, F, n, _ptr(out))
        return out

    # -- chained rounds ---------------------------------------------------------
    def homrec(self, ct, s_hat) -> torch.Tensor:
        """In place: ct uint64 [B][F][n+1][C] gains Delta * s_hat[b][c][f] on
        every b word, s_hat uint32 [B][C][F] (ensei_homrec); returns ct."""
        self._dev(ct, "ct", torch.uint64)
        self._dev(s_hat, "s_hat", torch.uint32)
        B, F, n1, Cc = tuple(ct.shape)
        if tuple(s_hat.shape) != (B, Cc, F):
            raise ValueError(f"s_hat must be [B][C][F] = {(B, Cc, F)}")
        self._call("ensei_homrec", _ptr(ct), _ptr(s_hat), B, Cc, F, n1 - 1)
        return ct

    def homrec_seeded(self, b_words, s_hat) -> torch.Tensor:
        """In place: seeded ciphertexts' b words uint64 [B][F][C] gain
        Delta * s_hat[b][c][f] (ensei_homrec_seeded); returns b_words."""
        self._dev(b_words, "b_words", torch.uint64)
        self._dev(s_hat, "s_hat", torch.uint32)
        B, F, Cc = tuple(b_words.shape)
        if tuple(s_hat.shape) != (B, Cc, F):
            raise ValueError(f"s_hat must be [B][C][F] = {(B, Cc, F)}")
        self._call("ensei_homrec_seeded", _ptr(b_words), _ptr(s_hat), B, Cc, F)
        return b_words

    def reshare(self, s_a, s_b, s_b_next, act: int, out=None) -> torch.Tensor:
        """The activation stand-in: f((s_a + s_b) mod p) - s_b_next mod p,
        f the identity (act 0) or the square (act 1) (ensei_reshare)."""
        for name, t in (("s_a", s_a), ("s_b", s_b), ("s_b_next", s_b_next)):
            self._dev(t, name, torch.uint32)
        if not (s_a.numel() == s_b.numel() == s_b_next.numel()):
            raise ValueError("the shares must hold the same number of residues")
        out = self._out(out, tuple(s_a.shape), torch.uint32)
        self._call("ensei_reshare", _ptr(s_a), _ptr(s_b), _ptr(s_b_next), s_a.numel(), int(act), _ptr(out))
        return out

    # -- HomConv ---------------------------------------------------------------
    def _hc_shapes(self, ct_in, Cout, r):
        B, F, n1, Cin = ct_in.shape  # word-major [B][F][n+1][Cin]
        if tuple(r.shape) != (B, Cout, F):
            raise ValueError(f"r must be [B][Cout][F] = {(B, Cout, F)}")
        return B, Cin, F, n1 - 1

    def homconv(self, ct_in, w_pack, r, Cout: int, out=None) -> torch.Tensor:
        """ct_in uint64 [B][F][n+1][Cin], packed W^, r uint32 [B][Cout][F] -> ct_out [B][F][n+1][Cout] (ensei_homconv)."""
        self._dev(ct_in, "ct_in", torch.uint64)
        self._dev(w_pack, "w_pack", torch.int8)
        self._dev(r, "r", torch.uint32)
        B, Cin, F, n = self._hc_shapes(ct_in, Cout, r)
        if w_pack.numel() < int(lib().ensei_wpack_bytes(Cout, Cin, F)):
            raise ValueError("w_pack is smaller than ensei_wpack_bytes(Cout, Cin, F)")
        out = self._out(out, (B, F, n + 1, Cout), torch.uint64)
        self._call("ensei_homconv", _ptr(ct_in), _ptr(w_pack), _ptr(r), B, Cin, Cout, F, n, _ptr(out))
        return out

    def homconv_seeded(self, b_in, n: int, seed_a: int, w_pack, r, Cout: int, ct_index0: int = 0,
                       out=None) -> torch.Tensor:
        """Seeded input: b words uint64 [B][F][Cin] and (seed_a, ct_index0) for
        the a-words of LWE dimension n -> ct_out [B][F][n+1][Cout], the same
        bits as homconv on the full ciphertexts (ensei_homconv_seeded)."""
        self._dev(b_in, "b_in", torch.uint64)
        self._dev(w_pack, "w_pack", torch.int8)
        self._dev(r, "r", torch.uint32)
        B, F, Cin = tuple(b_in.shape)
        if tuple(r.shape) != (B, Cout, F):
            raise ValueError(f"r must be [B][Cout][F] = {(B, Cout, F)}")
        if w_pack.numel() < int(lib().ensei_wpack_bytes(Cout, Cin, F)):
            raise ValueError("w_pack is smaller than ensei_wpack_bytes(Cout, Cin, F)")
        out = self._out(out, (B, F, n + 1, Cout), torch.uint64)
        self._call("ensei_homconv_seeded", _ptr(b_in), seed_a % 2**64, ct_index0 % 2**64, _ptr(w_pack), _ptr(r), B,
                   Cin, Cout, F, n, _ptr(out))
        return out

    def homconv_valu(self, ct_in, w_hat, r, out=None) -> torch.Tensor:
        """Same contraction from W^ uint32 [Cout][Cin][F] on the vector ALUs
        (ensei_bench_homconv_valu, in the comparison library libensei_bench.so)."""
        self._dev(ct_in, "ct_in", torch.uint64)
        self._dev(w_hat, "w_hat", torch.uint32)
        self._dev(r, "r", torch.uint32)
        Cout = w_hat.shape[0]
        B, Cin, F, n = self._hc_shapes(ct_in, Cout, r)
        if tuple(w_hat.shape) != (Cout, Cin, F):
            raise ValueError("w_hat must be [Cout][Cin][F]")
        out = self._out(out, (B, F, n + 1, Cout), torch.uint64)
        with torch.cuda.device(self.device):
            _check(bench_lib().ensei_bench_homconv_valu(self._h, _ptr(ct_in), _ptr(w_hat), _ptr(r), B, Cin, Cout, F, n,
                                                        _ptr(out), self._stream()), "ensei_bench_homconv_valu")
        return out


class Plan:
    """A batched plan (``ensei_plan``): a stack of independent secure
    convolutions captured as one HIP graph, HomConv of all layers in one
    persistent launch with an autotuned tile schedule.

    ``layers`` is a list of dicts with the shape (H, W, Cin, Cout, kh, kw, n,
    seed_a) and the device tensors w, x, s, e, r (inputs) and x_hat, ct_in,
    ct_out, m, s_a, s_b (written by every run); the plan keeps references to
    them. ``Plan.buffers(ctx, shape, ...)`` allocates the outputs."""

    _INPUTS = ("w", "x", "s", "e", "r")
    _OUTPUTS = ("x_hat", "ct_in", "ct_out", "m", "s_a", "s_b")

    def __init__(self, ctx: "Context", layers: list, tune_cache: str | None = None, seeded: bool = False):
        """seeded: seeded ciphertexts (ensei_plan_create_seeded); each layer's
        ct_in then holds only the b words, [batch][F][Cin]."""
        self.ctx = ctx
        self.layers = layers
        arr = (LayerDesc * len(layers))()
        for d, l in zip(arr, layers):
            B = l["x"].shape[0]
            for k in ("H", "W", "Cin", "Cout", "kh", "kw", "n"):
                setattr(d, k, int(l[k]))
            d.batch = int(B)
            d.seed_a = int(l["seed_a"]) & (2**64 - 1)
            dtypes = {"w": torch.int32, "x": torch.uint32, "s": torch.int8, "e": torch.int32, "r": torch.uint32,
                      "x_hat": torch.uint32, "ct_in": torch.uint64, "ct_out": torch.uint64, "m": torch.uint32,
                      "s_a": torch.uint32, "s_b": torch.uint32}
            H, W, Cin, Cout, n = (int(l[k]) for k in ("H", "W", "Cin", "Cout", "n"))
            F = H * W
            sizes = {"w": Cout * Cin * int(l["kh"]) * int(l["kw"]), "x": B * Cin * F, "s": n, "e": B * Cin * F,
                     "r": B * Cout * F, "x_hat": B * Cin * F, "ct_in": B * F * (1 if seeded else n + 1) * Cin,
                     "ct_out": B * F * (n + 1) * Cout, "m": B * Cout * F, "s_a": B * Cout * F, "s_b": B * Cout * F}
            for k in self._INPUTS + self._OUTPUTS:
                t = ctx._dev(l[k], k, dtypes[k])
                if t.numel() != sizes[k]:
                    raise ValueError(f"layer buffer {k} holds {t.numel()} elements, the shape needs {sizes[k]}")
                setattr(d, k, _ptr(t).value)
        h = C.c_void_p()
        cache = tune_cache.encode() if tune_cache else None
        with torch.cuda.device(ctx.device):
            name = "ensei_plan_create_seeded" if seeded else "ensei_plan_create"
            _check(getattr(lib(), name)(ctx._h, arr, len(layers), cache, C.byref(h)), name)
        self._h = h

    @staticmethod
    def buffers(ctx: "Context", H, W, Cin, Cout, n, batch, seeded: bool = False) -> dict:
        """Device outputs of one layer of a plan (seeded: ct_in holds the b words only)."""
        F = H * W
        return {
            "x_hat": ctx._empty((batch, Cin, F), torch.uint32),
            "ct_in": ctx._empty((batch, F, Cin) if seeded else (batch, F, n + 1, Cin), torch.uint64),
            "ct_out": ctx._empty((batch, F, n + 1, Cout), torch.uint64),
            "m": ctx._empty((batch, Cout, F), torch.uint32),
            "s_a": ctx._empty((batch, Cout, H, W), torch.uint32),
            "s_b": ctx._empty((batch, Cout, H, W), torch.uint32),
        }

    def run(self):
        """Enqueue one run of the captured graph on the current stream."""
        with torch.cuda.device(self.ctx.device):
            _check(lib().ensei_plan_run(self._h, self.ctx._stream()), "ensei_plan_run")

    def run_stage(self, stage: int):
        """Enqueue one stage (0 client NTT2D + Enc, 1 server HomConv, 2 Dec,
        INTT2D and the server's share) on the current stream."""
        with torch.cuda.device(self.ctx.device):
            _check(lib().ensei_plan_run_stage(self._h, int(stage), self.ctx._stream()), "ensei_plan_run_stage")

    def schedule(self) -> dict:
        sd = ScheduleDesc()
        _check(lib().ensei_plan_schedule(self._h, C.byref(sd)), "ensei_plan_schedule")
        return {"blocks": sd.blocks, "chunk": sd.chunk, "homconv_us": sd.homconv_us, "from_cache": bool(sd.from_cache),
                "shared_layers": sd.shared_layers, "own_layers": sd.own_layers, "branches": bool(sd.branches),
                "serial_us": sd.serial_us, "branches_us": sd.branches_us}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.ctx.device)
            lib().ensei_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A continuous-batching server (``ensei_server``) for secure-convolution
    requests of mixed shapes under a device-memory budget for their
    ciphertext state."""

    STATES = ("queued", "running", "done", "failed", "cancelled")

    def __init__(self, ctx: "Context", budget_bytes: int, nstreams: int = 4, max_batch: int = 16,
                 seeded: bool = False):
        """seeded: requests keep only the b words of their input ciphertexts
        (ensei_server_create_seeded)."""
        self.ctx = ctx
        h = C.c_void_p()
        name = "ensei_server_create_seeded" if seeded else "ensei_server_create"
        with torch.cuda.device(ctx.device):
            _check(getattr(lib(), name)(ctx._h, int(budget_bytes), nstreams, max_batch, C.byref(h)), name)
        self._h = h
        self._shapes = {}
        self._keep = {}  # ticket -> the request's tensors, kept alive until forget()

    @staticmethod
    def request_bytes(H, W, Cin, Cout, kh, kw, n) -> int:
        return int(lib().ensei_request_bytes(C.byref(ShapeDesc(H, W, Cin, Cout, kh, kw, n))))

    def add_shape(self, H, W, Cin, Cout, kh, kw, n, w: torch.Tensor) -> int:
        """Registers a shape with the server's filters w int32 [Cout][Cin][kh][kw]; returns its id."""
        self.ctx._dev(w, "w", torch.int32)
        if w.numel() != Cout * Cin * kh * kw:
            raise ValueError("w has the wrong size")
        sid = C.c_int()
        with torch.cuda.device(self.ctx.device):
            _check(lib().ensei_server_add_shape(self._h, C.byref(ShapeDesc(H, W, Cin, Cout, kh, kw, n)), _ptr(w),
                                                C.byref(sid)), "ensei_server_add_shape")
        self._shapes[sid.value] = (H, W, Cin, Cout, kh, kw, n)
        return sid.value

    def submit(self, shape_id: int, x, s, e, r, seed_a: int, s_a, s_b) -> int:
        """Queues one request (device tensors: x [Cin][H][W], s [n], e [Cin][F],
        r [Cout][F]; outputs s_a, s_b [Cout][H][W]). The request's kernels
        start after the work queued on the current stream so far, which may
        still be writing the inputs."""
        H, W, Cin, Cout, kh, kw, n = self._shapes[shape_id]
        F = H * W
        need = {"x": (x, torch.uint32, Cin * F), "s": (s, torch.int8, n), "e": (e, torch.int32, Cin * F),
                "r": (r, torch.uint32, Cout * F), "s_a": (s_a, torch.uint32, Cout * F),
                "s_b": (s_b, torch.uint32, Cout * F)}
        for k, (t, dt, cnt) in need.items():
            self.ctx._dev(t, k, dt)
            if t.numel() != cnt:
                raise ValueError(f"{k} holds {t.numel()} elements, the shape needs {cnt}")
        rq = RequestDesc(_ptr(x).value, _ptr(s).value, _ptr(e).value, _ptr(r).value, int(seed_a) & (2**64 - 1),
                         _ptr(s_a).value, _ptr(s_b).value, self.ctx._stream().value)
        t = C.c_uint64()
        _check(lib().ensei_server_submit(self._h, shape_id, C.byref(rq), C.byref(t)), "ensei_server_submit")
        self._keep[t.value] = (x, s, e, r, s_a, s_b)
        return t.value

    def cancel(self, ticket: int) -> None:
        """Cancels a queued request (it never runs) or marks a running one
        (reported cancelled when its batch ends); EnseiError(STATE) if the
        request has finished."""
        _check(lib().ensei_server_cancel(self._h, ticket), "ensei_server_cancel")

    def set_queue_limit(self, nbytes: int) -> None:
        """Caps the bytes of requests waiting for admission (0: no cap)."""
        _check(lib().ensei_server_set_queue_limit(self._h, int(nbytes)), "ensei_server_set_queue_limit")

    def clock(self) -> float:
        """Seconds since the server was created (the time base of poll())."""
        t = C.c_double()
        _check(lib().ensei_server_clock(self._h, C.byref(t)), "ensei_server_clock")
        return t.value

    def poll(self, ticket: int) -> dict:
        info = RequestInfo()
        _check(lib().ensei_server_poll(self._h, ticket, C.byref(info)), "ensei_server_poll")
        return {"state": self.STATES[info.state], "status": info.status, "t_submit": info.t_submit,
                "t_start": info.t_start, "t_done": info.t_done}

    def wait(self, ticket: int, timeout_ms: int = -1) -> None:
        _check(lib().ensei_server_wait(self._h, ticket, timeout_ms), "ensei_server_wait")

    def forget(self, ticket: int) -> None:
        _check(lib().ensei_server_forget(self._h, ticket), "ensei_server_forget")
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        si = ServerInfo()
        _check(lib().ensei_server_stats(self._h, C.byref(si)), "ensei_server_stats")
        return {k: int(getattr(si, k)) for k, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ensei_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
