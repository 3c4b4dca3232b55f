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


def rows_u64(t: torch.Tensor, flat_rows: np.ndarray) -> np.ndarray:
    """Gather rows of a uint64 [..., n+1] device tensor at flat row indices."""
    n1 = t.shape[-1]
    v = t.view(torch.int64).reshape(-1, n1)
    idx = torch.from_numpy(np.asarray(flat_rows, dtype=np.int64)).to(t.device)
    return host(v.index_select(0, idx)).view(np.uint64)


def oracle_ct_in_rows(orc, x_hat: np.ndarray, inp, b: int, f: int) -> np.ndarray:
    """The oracle's ciphertexts ct_in[b][:, f, :] ([Cin][n+1]) encrypted one by
    one with their global ciphertext index c = (b*Cin + i)*F + f."""
    S = inp.shape
    out = np.empty((S.Cin, S.n + 1), dtype=np.uint64)
    for i in range(S.Cin):
        c = (b * S.Cin + i) * S.F + f
        out[i] = orc.encrypt(
            x_hat[b, i, f : f + 1], inp.s, inp.e[b, i, f : f + 1], inp.seed_a, P, ct_index0=c
        )[0]
    return out


def oracle_ct_out_row(orc, ct_in_rows: np.ndarray, w_hat: np.ndarray, inp, b: int, o: int, f: int) -> np.ndarray:
    """The oracle's HomConv output row (b, o, f) from its own ct_in rows."""
    S = inp.shape
    ct = ct_in_rows.reshape(1, S.Cin, 1, S.n + 1)
    wf = np.ascontiguousarray(w_hat[:, :, f : f + 1])
    rf = np.ascontiguousarray(inp.r[b : b + 1, :, f : f + 1])
    return orc.homconv_select(ct, wf, rf, np.array([[0, o, 0]]), P)[0]
