"""Helpers for the GPU parity tests: host <-> device copies and oracle rows
computed one by one for sampled outputs of full-size runs."""
from __future__ import annotations

import numpy as np
import torch

P = 65537


def dev(a: np.ndarray, device: int = 0) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(f"cuda:{device}")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize(t.device)
    return t.cpu().numpy()


def ct_words(t: torch.Tensor, b: int, f: int, c: int) -> np.ndarray:
    """The n+1 words of ciphertext (b, c, f) of a word-major [B][F][n+1][C] tensor."""
    return host(t.view(torch.int64)[b, f, :, c].contiguous()).view(np.uint64)


def oracle_ct_in_rows(orc, x_hat: np.ndarray, inp, b: int, f: int) -> np.ndarray:
    """The oracle's ciphertexts of (b, :, f) ([Cin][n+1]), encrypted one by one
    with their ciphertext index q = (b*F + f)*Cin + i."""
    S = inp.shape
    out = np.empty((S.Cin, S.n + 1), dtype=np.uint64)
    for i in range(S.Cin):
        q = (b * S.F + f) * S.Cin + i
        out[i] = orc.encrypt(x_hat[b, i, f : f + 1], inp.s, inp.e[b, i, f : f + 1], inp.seed_a, P, ct_index0=q)[0]
    return out


def oracle_ct_out_row(orc, ct_in_rows: np.ndarray, w_hat: np.ndarray, inp, b: int, o: int, f: int) -> np.ndarray:
    """The oracle's HomConv output ciphertext (b, o, f) from its own input ciphertexts."""
    S = inp.shape
    ct = np.ascontiguousarray(ct_in_rows.T).reshape(1, 1, S.n + 1, S.Cin)
    wf = np.ascontiguousarray(w_hat[:, :, f : f + 1])
    rf = np.ascontiguousarray(inp.r[b : b + 1, :, f : f + 1])
    return orc.homconv_select(ct, wf, rf, np.array([[0, o, 0]]), P)[0]
