#!/usr/bin/env python3
"""Benchmark: the secure convolution hot path on one MI355X.

Headline (default): the CIFAR-shaped seven-layer stack, batch of 8 images
(layers (Cin, Cout, HxW) = (3,64,32), (64,64,32), (64,128,16), (128,128,16),
(128,256,8), (256,256,8), (256,512,4), 3x3 filters, LWE n = 1024, q = 2^64,
p = 65537), run as one batched plan: the server's filters are transformed and
packed once when the plan is created (setup), and a step is one run of the
plan with every input resident in HBM:
  client   x^ = NTT2D(x); ct_in = Enc(x^)                 stage 0
  server   ct_out = HomConv(ct_in, W^) + Delta r          stage 1
  client   m = Dec(ct_out); s_A = INTT2D(m)               stage 2
  server   s_B = INTT2D(-r)                               stage 2
each stage a captured HIP graph over all seven layers, timed with HIP events
on the stream it runs on.

Prints ONE JSON line: the metric is whole-step throughput in ciphertext-MACs
per second (B*Cout*Cin*F scalar x ciphertext multiply-accumulates per layer,
each n+1 words), with the roofline of the HomConv stage (algorithmic HBM bytes
over its event-timed duration) and the CPU oracle's rate on the host cores.
`--workload <layer>` times one layer's whole step through the single calls
instead (the former headline, the 32x32 64 -> 64 layer, is one of the extras).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
DEFAULT_WORKLOAD = "stack8"
LAYER_WORKLOAD = "conv32x32_c64to64_k3_n1024"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "homconv_traffic.json")
STACK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "homconv_traffic_stack8.json")
# 32-bit integer vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HOMCONV_SRC = os.path.join(ROOT, "paper_2003_05328_amd", "csrc", "homconv.hip")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    help="stack8 (the seven-layer stack, batch 8, as a plan) or one layer name of configs.WORKLOADS")
    ap.add_argument("--homconv", choices=["mfma", "valu"], default="mfma",
                    help="HomConv kernel: matrix-core (ensei_homconv) or vector-ALU comparison (ensei_homconv_valu)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the CPU-oracle baseline (0: OMP_NUM_THREADS, else the usable cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the NTT2D throughput and the batched conv-stack comparison")
    ap.add_argument("--stack-reps", type=int, default=5)
    ap.add_argument("--serve", action="store_true",
                    help="only the serving sweep (Poisson arrivals of mixed-shape requests), one JSON line")
    ap.add_argument("--serve-rates", default="250,500,750,1000,1250,1500,2000", help="arrival rates, requests/s")
    ap.add_argument("--serve-requests", type=int, default=4000, help="requests per rate")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-streams", type=int, default=2, help="streams of the continuous-batching server")
    ap.add_argument("--serve-max-batch", type=int, default=4, help="requests per batch")
    ap.add_argument("--seeded", action="store_true",
                    help="only the main workload's step with seeded ciphertexts, one JSON line")
    ap.add_argument("--chained", action="store_true",
                    help="only two protocol rounds chained by HomRec (the stack's 32x32 pair), one JSON line")
    ap.add_argument("--packed", action="store_true",
                    help="only the packed (BFV) instantiation on Table 4's benchmarks, one JSON line")
    ap.add_argument("--packed-batch", type=int, default=64)
    ap.add_argument("--ntt", action="store_true",
                    help="only the NTT2D weight-batch measurements (the ntt2d entry of the default line)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="run only a plain 1 GiB read + 1 GiB write elementwise kernel (counter calibration)")
    return ap.parse_args()


def probe_copy(reps: int = 3):
    """A plain elementwise kernel of known traffic: reads and writes 1 GiB.
    rocprofv3's FETCH_SIZE / WRITE_SIZE on it calibrate the HBM counters."""
    import torch

    n = 1 << 28  # int32 elements = 1 GiB
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "launches": reps}), flush=True)


def homconv_bytes(S, pack_bytes: int) -> int:
    """Algorithmic HBM bytes of one HomConv launch: ct_in read once, ct_out
    written once, the packed weights and the masks read once."""
    return 8 * (S.n + 1) * S.F * S.B * (S.Cin + S.Cout) + pack_bytes + 4 * S.B * S.Cout * S.F


def traffic_entry(path: str = TRAFFIC_FILE, workload: str = None, kernel: str = None):
    """Measured HBM bytes per launch (or per plan stage) from rocprofv3
    counters, if they were taken on the current HomConv source (and, when
    given, on this workload and kernel); else None."""
    from paper_2003_05328_amd.profile_summary import code_digest

    try:
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("code_sha256") != code_digest(HOMCONV_SRC):
            return None
        if workload is not None and rec.get("workload") != workload:
            return None
        if kernel is not None and not rec.get("kernel", "").startswith(kernel):
            return None
        return int(rec["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def homconv_kernel_name(S, seeded: bool = False) -> str:
    """The kernel ensei_homconv launches for one layer, by the library's
    launch rule (homconv.hip): the deep kernel for Cin >= 48 when its LDS
    layout fits (Cin <= 256, two or more row tiles and, for plain input, at
    least four (row tile, K step) pairs per block); else the narrow kernel
    for Cin <= 8; else the streaming kernel."""
    n_ks, n_ot = -(-S.Cin // 64), -(-S.Cout // 64)
    if S.Cin >= 48 and n_ks <= 4 and n_ot >= 2 and (seeded or n_ot * n_ks >= 4):
        n_dma = 0 if seeded else -(-(32 * S.Cin * 8) // 1024)
        n_mask = 2 * ((n_ot + 1) // 2) * 64
        lds = n_ks * 8 * 2048 + n_dma * 1024 + 2 * n_mask * 4 + (64 if S.Cin % 8 else 0)
        if lds <= 160 * 1024:
            return "homconv_deep_kernel"
    if S.Cin <= 8:
        return "homconv_narrow_kernel"
    return "homconv_mfma_kernel"


MFMA_I8_PEAK_MACS = 2.5e15  # dense i8 multiply-accumulates per second (5.0 POP/s)


def homconv_layers(ctx, warm: int = 10, reps: int = 10):
    """HomConv alone on every distinct workload layer shape (random words: the
    kernels' cost does not depend on values), timed after `warm` launches as
    the mean of `reps`: the algorithmic HBM rate, and the i8 multiply-
    accumulate rate (21 per word-MAC) against the dense matrix-core peak; and
    the same layer's seeded HomConv time (b words in, a-words regenerated)."""
    import torch
    from paper_2003_05328_amd import configs

    P = configs.P
    rows = []
    for name, S in configs.WORKLOADS.items():
        if name.endswith("_hidden") or S.binary:  # same HomConv shape as another entry
            continue
        dv = "cuda:0"
        ct = torch.empty((S.B, S.F, S.n + 1, S.Cin), dtype=torch.int64, device=dv).random_().view(torch.uint64)
        w = torch.randint(0, P, (S.Cout, S.Cin, S.F), dtype=torch.int32, device=dv).view(torch.uint32)
        r = torch.randint(0, P, (S.B, S.Cout, S.F), dtype=torch.int32, device=dv).view(torch.uint32)
        pack = ctx.pack_weights(w)
        out = torch.empty((S.B, S.F, S.n + 1, S.Cout), dtype=torch.uint64, device=dv)
        for _ in range(warm):
            ctx.homconv(ct, pack, r, S.Cout, out=out)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            ctx.homconv(ct, pack, r, S.Cout, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        # the same layer on seeded input (b words only, a-words regenerated)
        bw = torch.empty((S.B, S.F, S.Cin), dtype=torch.int64, device=dv).random_().view(torch.uint64)
        for _ in range(warm):
            ctx.homconv_seeded(bw, S.n, 12345, pack, r, S.Cout, out=out)
        ev[0].record()
        for _ in range(reps):
            ctx.homconv_seeded(bw, S.n, 12345, pack, r, S.Cout, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        us_seeded = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        nbytes = homconv_bytes(S, int(pack.numel()))
        word_macs = S.B * S.Cout * S.Cin * S.F * (S.n + 1)
        i8 = 21 * word_macs / (us * 1e-6)
        rows.append({"layer": name, "us": us, "algorithmic_bytes": nbytes,
                     "hbm_gbs": nbytes / (us * 1e-6) / 1e9, "frac_hbm": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "word_mac_per_byte": word_macs / nbytes, "i8_mac_per_s": i8, "frac_mfma": i8 / MFMA_I8_PEAK_MACS,
                     "seeded_us": us_seeded})
        del ct, w, r, pack, out, bw
        torch.cuda.empty_cache()
    return rows


def ntt_line_ops(L: int) -> int:
    """Integer ALU ops of one radix-2 transform of length L: per butterfly 10
    int32 ops with a twiddle (add, reduce, subtract, Shoup multiply), 6
    without (j = 0)."""
    ops, m = 0, L
    while m >= 2:
        ops += (L // m) * (6 + 10 * (m // 2 - 1))
        m //= 2
    return ops


def ntt_throughput(ctx, batches, reps: int = 5):
    """NTT2D on weight-preparation batches (one launch per (grids, H, W) entry),
    each repetition after reading a 1 GiB buffer through the caches so that
    the grids come from HBM (a read, not a read-modify-write: a written
    buffer would leave the caches full of dirty lines whose write-back then
    lands inside the timed launch): points/s, the algorithmic HBM rate
    (4 bytes read and 4 written per point) and the integer ALU rate, each
    against its peak. batches: list of (grids, H, W)."""
    import numpy as np
    import torch

    dv = "cuda:0"
    flush = torch.ones(1 << 27, dtype=torch.int64, device=dv)  # summed in its own type: no converted copy
    sink = torch.zeros((), dtype=torch.int64, device=dv)
    bufs = []
    for grids, H, W in batches:
        x = torch.randint(0, 65537, (grids, H, W), dtype=torch.int32, device=dv).view(torch.uint32)
        bufs.append((x, torch.empty((grids, H * W), dtype=torch.uint32, device=dv), H, W))
    for x, out, H, W in bufs:
        ctx.ntt2d(x, out=out)
    times = []
    for _ in range(reps):
        t = 0.0
        for x, out, H, W in bufs:
            sink += flush.sum()  # 1 GiB read: evicts the grids from the last-level cache
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            ctx.ntt2d(x, out=out)
            ev[1].record()
            torch.cuda.synchronize()
            t += ev[0].elapsed_time(ev[1]) * 1e3
        times.append(t)
    us = float(np.median(times))
    pts = sum(g * H * W for g, H, W in batches)
    ops = sum(g * (H * ntt_line_ops(W) + W * ntt_line_ops(H)) for g, H, W in batches)
    gbs = 8 * pts / (us * 1e-6) / 1e9
    tops = ops / (us * 1e-6) / 1e12
    del flush, bufs
    torch.cuda.empty_cache()
    return {"launches": [f"{g}x{H}x{W}" for g, H, W in batches], "points": pts, "avg_us": us,
            "points_per_s": pts / (us * 1e-6), "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "bytes_per_point": 8, "cache": "flushed (1 GiB read) before each launch",
            "alu": {"achieved": tops, "peak": ALU_PEAK_TOPS, "unit": "T int32 op/s", "frac": tops / ALU_PEAK_TOPS,
                    "ops": ops}}


def seeded_step(ctx, S, inp, steps: int, warmup: int):
    """The whole step of the main workload with seeded ciphertexts (Sec. 5.1:
    the ciphertexts' public constants are generated offline): Enc keeps only
    the b words and HomConv regenerates the a-words. Checked like the main
    step (exact decryption of every output)."""
    import numpy as np
    import torch
    from paper_2003_05328_amd import configs
    from paper_2003_05328_amd.ensei import lib

    P = configs.P
    dv = "cuda:0"
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dv)
    x, w, s, e, r = d(inp.x), d(inp.w), d(inp.s), d(inp.e), d(inp.r)
    pack_bytes = int(lib().ensei_wpack_bytes(S.Cout, S.Cin, S.F))
    w_hat = torch.empty((S.Cout, S.Cin, S.F), dtype=torch.uint32, device=dv)
    pack = torch.empty((pack_bytes,), dtype=torch.int8, device=dv)
    x_hat = torch.empty((S.B, S.Cin, S.F), dtype=torch.uint32, device=dv)
    b_in = torch.empty((S.B, S.F, S.Cin), dtype=torch.uint64, device=dv)
    ct_out = torch.empty((S.B, S.F, S.n + 1, S.Cout), dtype=torch.uint64, device=dv)
    m = torch.empty((S.B, S.Cout, S.F), dtype=torch.uint32, device=dv)
    s_a = torch.empty((S.B, S.Cout, S.H, S.W), dtype=torch.uint32, device=dv)
    s_b = torch.empty((S.B, S.Cout, S.H, S.W), dtype=torch.uint32, device=dv)
    names = ["weight_prep", "pack_weights", "ntt2d", "encrypt_seeded", "homconv_seeded", "decrypt", "intt2d",
             "server_share"]

    def step(ev=None):
        mark = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
        mark(0)
        ctx.weight_prep(w, S.H, S.W, out=w_hat)
        mark(1)
        ctx.pack_weights(w_hat, out=pack)
        mark(2)
        ctx.ntt2d(x, out=x_hat)
        mark(3)
        ctx.encrypt_seeded(x_hat, s, e, inp.seed_a, out=b_in)
        mark(4)
        ctx.homconv_seeded(b_in, S.n, inp.seed_a, pack, r, S.Cout, out=ct_out)
        mark(5)
        ctx.decrypt(ct_out, s, out=m)
        mark(6)
        ctx.intt2d(m, S.H, S.W, out=s_a)
        mark(7)
        ctx.server_share(r, S.H, S.W, out=s_b)
        mark(8)

    for _ in range(warmup):
        step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(events[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    xh = x_hat.cpu().numpy().astype(np.int64)
    wh = w_hat.cpu().numpy().astype(np.int64)
    ok = bool(np.array_equal(m.cpu().numpy().astype(np.int64), (np.einsum("oif,bif->bof", wh, xh) + inp.r) % P))
    kernels_us = {nm: float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in events])) * 1e3
                  for i, nm in enumerate(names)}
    # the client's errors drawn on the device instead of on the host
    e_dev = torch.empty((S.B, S.Cin, S.F), dtype=torch.int32, device=dv)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(20):
        ctx.sample_errors(inp.seed_a ^ 0x5EED, S.B, S.Cin, S.F, out=e_dev)
    ev[1].record()
    torch.cuda.synchronize()
    kernels_us["sample_errors (device-drawn e, not in the step)"] = ev[0].elapsed_time(ev[1]) * 1e3 / 20
    hc_us = kernels_us["homconv_seeded"]
    # algorithmic bytes of the seeded HomConv: b words in, ct_out out, weights, masks
    hc_bytes = 8 * S.F * S.B * (S.Cin + (S.n + 1) * S.Cout) + pack_bytes + 4 * S.B * S.Cout * S.F
    macs = S.B * S.Cout * S.Cin * S.F
    return {"ms_per_step": ms, "ct_mac_per_s": macs / (ms * 1e-3), "kernels_us": kernels_us,
            "homconv_seeded": {"algorithmic_bytes": hc_bytes, "avg_us": hc_us,
                               "achieved_gbs": hc_bytes / (hc_us * 1e-6) / 1e9,
                               "frac_hbm": hc_bytes / (hc_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
            "verified": ok}


def chained(ctx, reps: int, seed: int, act: int = 1):
    """Two rounds of Fig. 2 chained on the device: the CIFAR stack's 32x32
    3 -> 64 and 64 -> 64 layers (batch 8, n = 1024), joined by the activation
    stand-in (square), the client's NTT2D and Enc of its new share, and the
    server's HomRec with its transformed share. Each pass includes both layers'
    filter preparation. Checked on the pass's own intermediates: round 0's and
    round 1's plaintexts, and the shares after the activation."""
    import numpy as np
    import torch
    from paper_2003_05328_amd import configs, synth

    P = configs.P
    S0 = configs.WORKLOADS["stack8_L1_32x32_c3to64"]
    S1 = configs.WORKLOADS["stack8_L2_32x32_c64to64"]
    inp0, inp1 = synth.generate(S0, P, seed), synth.generate(S1, P, seed + 1)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    x0, w0, s0, e0, r0 = d(inp0.x), d(inp0.w), d(inp0.s), d(inp0.e.reshape(S0.B, S0.Cin, S0.F)), d(inp0.r)
    w1, s1, e1, r1 = d(inp1.w), d(inp1.s), d(inp1.e.reshape(S1.B, S1.Cin, S1.F)), d(inp1.r)
    s_b1 = d(synth.uniform_u32(seed + 2, (S1.B, S1.Cin, S1.H, S1.W), P))
    names = ["round0", "reshare", "client_ntt_enc", "homrec", "round1"]
    keep = {}

    def pass_(ev=None):
        mark = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
        mark(0)
        x_hat0 = ctx.ntt2d(x0)
        w_hat0 = ctx.weight_prep(w0, S0.H, S0.W)
        ct0 = ctx.encrypt(x_hat0, s0, e0, inp0.seed_a)
        m0 = ctx.decrypt(ctx.homconv(ct0, ctx.pack_weights(w_hat0), r0, S0.Cout), s0)
        s_a0 = ctx.intt2d(m0, S0.H, S0.W)
        s_b0 = ctx.server_share(r0, S0.H, S0.W)
        mark(1)
        s_a1 = ctx.reshare(s_a0, s_b0, s_b1, act)
        mark(2)
        x_hat1 = ctx.ntt2d(s_a1)
        ct1 = ctx.encrypt(x_hat1, s1, e1, inp1.seed_a)
        sb_hat = ctx.ntt2d(s_b1)
        mark(3)
        ctx.homrec(ct1, sb_hat)
        mark(4)
        w_hat1 = ctx.weight_prep(w1, S1.H, S1.W)
        m1 = ctx.decrypt(ctx.homconv(ct1, ctx.pack_weights(w_hat1), r1, S1.Cout), s1)
        s_a = ctx.intt2d(m1, S1.H, S1.W)
        s_b = ctx.server_share(r1, S1.H, S1.W)
        mark(5)
        keep.update(x_hat0=x_hat0, w_hat0=w_hat0, m0=m0, s_a0=s_a0, s_b0=s_b0, s_a1=s_a1, x_hat1=x_hat1,
                    sb_hat=sb_hat, w_hat1=w_hat1, m1=m1, s_a=s_a, s_b=s_b)

    for _ in range(2):
        pass_()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        pass_(events[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    part_us = {nm: float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in events])) * 1e3 for i, nm in enumerate(names)}
    # the same two rounds on seeded ciphertexts: Enc keeps the b words, HomRec
    # adds the server's share to them, HomConv regenerates the a-words
    keep_s = {}

    def pass_seeded():
        x_hat0 = ctx.ntt2d(x0)
        bw0 = ctx.encrypt_seeded(x_hat0, s0, e0, inp0.seed_a)
        m0 = ctx.decrypt(ctx.homconv_seeded(bw0, S0.n, inp0.seed_a, ctx.pack_weights(ctx.weight_prep(w0, S0.H, S0.W)),
                                            r0, S0.Cout), s0)
        s_a1 = ctx.reshare(ctx.intt2d(m0, S0.H, S0.W), ctx.server_share(r0, S0.H, S0.W), s_b1, act)
        bw1 = ctx.encrypt_seeded(ctx.ntt2d(s_a1), s1, e1, inp1.seed_a)
        ctx.homrec_seeded(bw1, ctx.ntt2d(s_b1))
        m1 = ctx.decrypt(ctx.homconv_seeded(bw1, S1.n, inp1.seed_a, ctx.pack_weights(ctx.weight_prep(w1, S1.H, S1.W)),
                                            r1, S1.Cout), s1)
        keep_s.update(m1=m1, s_a=ctx.intt2d(m1, S1.H, S1.W))

    for _ in range(2):
        pass_seeded()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pass_seeded()
    torch.cuda.synchronize()
    ms_seeded = (time.perf_counter() - t0) * 1e3 / reps
    seeded_same = torch.equal(keep_s["m1"], keep["m1"]) and torch.equal(keep_s["s_a"], keep["s_a"])

    h = {k: v.cpu().numpy().astype(np.int64) for k, v in keep.items()}
    ok0 = np.array_equal(h["m0"], (np.einsum("oif,bif->bof", h["w_hat0"], h["x_hat0"]) + inp0.r) % P)
    y0 = (h["s_a0"] + h["s_b0"]) % P
    ok_act = np.array_equal((h["s_a1"] + s_b1.cpu().numpy()) % P, y0 if act == 0 else y0 * y0 % P)
    u_hat = (h["x_hat1"] + h["sb_hat"]) % P  # the transform of the reconstructed activation
    ok1 = np.array_equal(h["m1"], (np.einsum("oif,bif->bof", h["w_hat1"], u_hat) + inp1.r) % P)
    macs = S0.B * S0.Cout * S0.Cin * S0.F + S1.B * S1.Cout * S1.Cin * S1.F
    n_ct = S1.B * S1.Cin * S1.F
    hr_bytes = n_ct * (4 + 8 + 8)  # the share read, each b word read and written
    return {"workload": "CIFAR stack layers 1-2 chained: 32x32 3->64 then 64->64, 3x3, n=1024, batch 8, "
                        f"activation {'square' if act else 'identity'} (stand-in, in the clear)",
            "ms_per_pass": ms, "ct_mac_per_s": macs / (ms * 1e-3), "parts_us": part_us,
            "homrec": {"ciphertexts": n_ct, "bytes": hr_bytes, "us": part_us["homrec"],
                       "achieved_gbs": hr_bytes / (part_us["homrec"] * 1e-6) / 1e9},
            "seeded": {"ms_per_pass": ms_seeded, "ct_mac_per_s": macs / (ms_seeded * 1e-3),
                       "bit_exact_vs_unseeded": bool(seeded_same)},
            "bit_exact": bool(ok0 and ok_act and ok1 and seeded_same)}


def stack_batched(ctx, reps: int, seed: int):
    """The seven-layer conv stack (batch of 8 images) as one batched plan (one
    graph, one persistent HomConv launch, tuned schedule) against plain
    execution one request at a time (each image's layer a secure convolution
    of its own, through the single calls) and against the same batch-8 layers
    one after another through the single calls; all bit-exact."""
    import numpy as np
    import torch

    from paper_2003_05328_amd import configs, synth
    from paper_2003_05328_amd.ensei import Plan

    shapes = configs.stack_shapes(B=8)
    P = configs.P
    layers, packs = [], []
    for i, S in enumerate(shapes):
        inp = synth.generate(S, P, seed + 1000 + i)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
        l = {"H": S.H, "W": S.W, "Cin": S.Cin, "Cout": S.Cout, "kh": S.kh, "kw": S.kw, "n": S.n,
             "seed_a": inp.seed_a, "w": d(inp.w), "x": d(inp.x), "s": d(inp.s), "e": d(inp.e), "r": d(inp.r)}
        l.update(Plan.buffers(ctx, S.H, S.W, S.Cin, S.Cout, S.n, S.B))
        layers.append(l)
    t0 = time.perf_counter()
    plan = Plan(ctx, layers)
    create_s = time.perf_counter() - t0
    sched = plan.schedule()
    # one-at-a-time baseline: the same kernels, single calls, filters prepared beforehand
    seq = []
    for S, l in zip(shapes, layers):
        pack = ctx.pack_weights(ctx.weight_prep(l["w"], S.H, S.W))
        seq.append({k: torch.empty_like(l[k]) for k in ("x_hat", "ct_in", "ct_out", "m", "s_a", "s_b")})
        packs.append(pack)

    def sequential():
        for S, l, o, pk in zip(shapes, layers, seq, packs):
            ctx.ntt2d(l["x"], out=o["x_hat"].view(S.B * S.Cin, S.F))
            ctx.encrypt(o["x_hat"], l["s"], l["e"], l["seed_a"], out=o["ct_in"])
            ctx.homconv(o["ct_in"], pk, l["r"], S.Cout, out=o["ct_out"])
            ctx.decrypt(o["ct_out"], l["s"], out=o["m"])
            ctx.intt2d(o["m"].view(S.B * S.Cout, S.F), S.H, S.W, out=o["s_a"].view(S.B * S.Cout, S.F))
            ctx.server_share(l["r"].view(S.B * S.Cout, S.F), S.H, S.W, out=o["s_b"].view(S.B * S.Cout, S.F))

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
        return float(np.median(ts))

    def one_image_at_a_time():
        """Every layer of every image as its own secure convolution (B = 1,
        the same kernels); image b encrypts with the ciphertext indices of
        its place in the batch, so the words equal the batched ones."""
        for S, l, o, pk in zip(shapes, layers, seq, packs):
            for b in range(S.B):
                xh = o["x_hat"][b:b + 1]
                ctx.ntt2d(l["x"][b:b + 1], out=xh.view(S.Cin, S.F))
                ctx.encrypt(xh, l["s"], l["e"][b:b + 1], l["seed_a"], ct_index0=b * S.F * S.Cin,
                            out=o["ct_in"][b:b + 1])
                ctx.homconv(o["ct_in"][b:b + 1], pk, l["r"][b:b + 1], S.Cout, out=o["ct_out"][b:b + 1])
                ctx.decrypt(o["ct_out"][b:b + 1], l["s"], out=o["m"][b:b + 1])
                ctx.intt2d(o["m"][b].view(S.Cout, S.F), S.H, S.W, out=o["s_a"][b].view(S.Cout, S.F))
                ctx.server_share(l["r"][b].view(S.Cout, S.F), S.H, S.W, out=o["s_b"][b].view(S.Cout, S.F))

    plan_ms = timed(plan.run)
    one_ms = timed(one_image_at_a_time)
    same_one = all(torch.equal(l[k], o[k]) for l, o in zip(layers, seq) for k in ("ct_in", "ct_out", "m", "s_a", "s_b"))
    seq_ms = timed(sequential)
    same = all(torch.equal(l[k], o[k]) for l, o in zip(layers, seq) for k in ("ct_in", "ct_out", "m", "s_a", "s_b"))
    macs = sum(S.B * S.Cout * S.Cin * S.F for S in shapes)
    hc_bytes = sum(8 * (S.n + 1) * S.F * S.B * (S.Cin + S.Cout) for S in shapes)
    plan.close()
    del seq
    torch.cuda.empty_cache()
    # the same stack on seeded ciphertexts (b words only on the input side)
    sl = []
    for S, l in zip(shapes, layers):
        d = {k: l[k] for k in ("H", "W", "Cin", "Cout", "kh", "kw", "n", "seed_a", "w", "x", "s", "e", "r")}
        d.update(Plan.buffers(ctx, S.H, S.W, S.Cin, S.Cout, S.n, S.B, seeded=True))
        sl.append(d)
    splan = Plan(ctx, sl, seeded=True)
    seeded_ms = timed(splan.run)
    seeded_same = all(torch.equal(a[k], b[k]) for a, b in zip(sl, layers) for k in ("ct_out", "m", "s_a", "s_b"))
    seeded_same = seeded_same and all(torch.equal(a["ct_in"], b["ct_in"][:, :, S.n, :])
                                      for S, a, b in zip(shapes, sl, layers))
    seeded_sched = splan.schedule()
    splan.close()
    return {
        "workload": "stack8: 7 layers (3,64,32),(64,64,32),(64,128,16),(128,128,16),(128,256,8),(256,256,8),"
                    "(256,512,4), 3x3, n=1024, batch 8",
        "ct_macs": macs,
        "batched_ms": plan_ms,
        "one_image_at_a_time_ms": one_ms,
        "sequential_ms": seq_ms,
        "batched_ct_mac_per_s": macs / (plan_ms * 1e-3),
        "one_image_at_a_time_ct_mac_per_s": macs / (one_ms * 1e-3),
        "sequential_ct_mac_per_s": macs / (seq_ms * 1e-3),
        "speedup_vs_one_image_at_a_time": one_ms / plan_ms,
        "speedup": seq_ms / plan_ms,
        "homconv_schedule": sched,
        "homconv_ct_bytes": hc_bytes,
        "plan_create_s": create_s,
        "bit_exact_vs_sequential": bool(same and same_one),
        "seeded": {"batched_ms": seeded_ms, "ct_mac_per_s": macs / (seeded_ms * 1e-3),
                   "homconv_schedule": seeded_sched, "bit_exact_vs_unseeded": bool(seeded_same)},
    }


def serving(ctx, rates, n_req: int, budget_gb: float, seed: int, nstreams: int = 2, max_batch: int = 4,
            seeded_rates=None, p99_target_ms: float = 25.0):
    """Secure-convolution requests of mixed shapes (one image each: pick one of
    the four workload families uniformly, then one of its layers) arriving as
    an open-loop Poisson process, served with continuous batching under a
    ciphertext budget; against sequential plain execution on the same GPU
    (one stream, batches of one request, first come first served) under the
    same arrivals. Latency runs from each request's scheduled arrival time
    (so a submitter that falls behind does not hide queueing) to its
    completion, in the server's clock. Every result is compared with the same
    request computed alone."""
    import threading

    import numpy as np
    import torch

    from paper_2003_05328_amd import configs, synth
    from paper_2003_05328_amd.ensei import Server

    P = configs.P
    W = configs.WORKLOADS
    families = [
        [W["conv16x16_c3to8_k3_n512"]],
        [W["conv32x32_c64to64_k3_n1024"], W["conv32x32_c64to64_k3_n1024_hidden"]],
        [S for k, S in W.items() if k.startswith("stack8_L")],
        [W["conv64x64(56)_c64to64_k3_n1024"], W["conv128x128_c3to64_k7_n1024"]],
    ]
    budget = int(budget_gb * (1 << 30))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    RING = 64

    def setup(server):
        fams = []
        for fi, fam in enumerate(families):
            lst = []
            for li, S0 in enumerate(fam):
                S = synth.LayerShape(S0.H, S0.W, S0.Cin, S0.Cout, S0.kh, S0.kw, S0.n, 1, S0.img_h, S0.img_w,
                                     S0.hidden, S0.binary)
                base = synth.generate(S, P, seed + 100 * fi + li)
                w = d(base.w)
                sid = server.add_shape(S.H, S.W, S.Cin, S.Cout, S.kh, S.kw, S.n, w)
                sets = []
                for j in range(2):
                    inp = synth.generate(S, P, seed + 10000 + 100 * fi + 10 * li + j)
                    sets.append({"x": d(inp.x[0]), "s": d(inp.s), "e": d(inp.e[0]), "r": d(inp.r[0]),
                                 "seed_a": inp.seed_a})
                ring = [(torch.empty((S.Cout, S.H, S.W), dtype=torch.uint32, device="cuda:0"),
                         torch.empty((S.Cout, S.H, S.W), dtype=torch.uint32, device="cuda:0")) for _ in range(RING)]
                lst.append({"S": S, "sid": sid, "sets": sets, "ring": ring, "free": list(range(RING)),
                            "ref": [None, None]})
            fams.append(lst)
        return fams

    def draw(g, n):
        out = []
        for _ in range(n):
            fi = int(g.integers(len(families)))
            li = int(g.integers(len(families[fi])))
            out.append((fi, li, int(g.integers(2))))
        return out

    def run(server, fams, plan, rate):
        """plan: list of (family, layer, set); Poisson arrivals at `rate`."""
        lock = threading.Condition()
        tickets = []
        done_flag = [False]
        ok = [True]
        times = []

        def collector():
            k = 0
            while True:
                with lock:
                    while k >= len(tickets) and not done_flag[0]:
                        lock.wait()
                    if k >= len(tickets):
                        return
                    t, L, j, slot, arrival = tickets[k]
                server.wait(t)
                info = server.poll(t)
                s_a, s_b = L["ring"][slot]
                same = torch.equal(s_a, L["ref"][j][0]) and torch.equal(s_b, L["ref"][j][1])
                server.forget(t)
                with lock:
                    ok[0] = ok[0] and same and info["state"] == "done"
                    times.append((arrival, info["t_submit"], info["t_start"], info["t_done"]))
                    L["free"].append(slot)
                    lock.notify_all()
                k += 1

        th = threading.Thread(target=collector)
        th.start()
        g = np.random.default_rng(seed + 7)
        gaps = g.exponential(1.0 / rate, size=len(plan))
        c0 = server.clock()  # the server's clock at t0: scheduled arrivals in its time base
        t0 = time.perf_counter()
        due = 0.0
        for (fi, li, j), gap in zip(plan, gaps):
            L = fams[fi][li]
            due += gap
            while time.perf_counter() - t0 < due:
                pass
            with lock:
                while not L["free"]:
                    lock.wait()
                slot = L["free"].pop()
            io = L["sets"][j]
            s_a, s_b = L["ring"][slot]
            t = server.submit(L["sid"], io["x"], io["s"], io["e"], io["r"], io["seed_a"], s_a, s_b)
            with lock:
                tickets.append((t, L, j, slot, c0 + due))
                lock.notify_all()
        with lock:
            done_flag[0] = True
            lock.notify_all()
        th.join()
        ts = np.array(times)
        lat = (ts[:, 3] - ts[:, 0]) * 1e3
        span = ts[:, 3].max() - ts[:, 0].min()
        return {"offered_req_s": rate, "requests": len(plan), "throughput_req_s": len(plan) / span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()),
                "submit_lag_p99_ms": float(np.percentile((ts[:, 1] - ts[:, 0]) * 1e3, 99)),
                "queue_p99_ms": float(np.percentile((ts[:, 2] - ts[:, 1]) * 1e3, 99)), "bit_exact": bool(ok[0])}

    def sweep(server, fams, plan, rs, label):
        out = []
        for r in rs:
            out.append(run(server, fams, plan, r))
            x = out[-1]
            # a progress line per rate (a long sweep is otherwise silent for minutes)
            print(f"serving {label}: {r:g} req/s offered, {x['throughput_req_s']:.0f} served, p50 {x['p50_ms']:.2f} "
                  f"ms, p99 {x['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
        return out

    g = np.random.default_rng(seed)
    plan = draw(g, n_req)
    server = Server(ctx, budget, nstreams=nstreams, max_batch=max_batch)
    fams = setup(server)
    # references: each input set alone, through the server one at a time
    for lst in fams:
        for L in lst:
            for j, io in enumerate(L["sets"]):
                s_a, s_b = torch.empty_like(L["ring"][0][0]), torch.empty_like(L["ring"][0][1])
                t = server.submit(L["sid"], io["x"], io["s"], io["e"], io["r"], io["seed_a"], s_a, s_b)
                server.wait(t)
                server.forget(t)
                L["ref"][j] = (s_a, s_b)
    torch.cuda.synchronize()
    batched = sweep(server, fams, plan, rates, "continuous batching")
    st = server.stats()
    server.close()
    refs = [[L["ref"] for L in lst] for lst in fams]

    def with_refs(srv):
        f = setup(srv)
        for lst, rl in zip(f, refs):
            for L, r in zip(lst, rl):
                L["ref"] = r
        return f

    seeded = []
    if seeded_rates:
        # requests keep only the b words of their input ciphertexts
        server = Server(ctx, budget, nstreams=nstreams, max_batch=max_batch, seeded=True)
        seeded = sweep(server, with_refs(server), plan, seeded_rates, "seeded")
        server.close()
    # sequential plain execution on the same GPU: one stream, one request at a
    # time, first come first served, the same open-loop arrivals
    seq_server = Server(ctx, budget, nstreams=1, max_batch=1)
    sequential = sweep(seq_server, with_refs(seq_server), plan, rates, "sequential")
    seq_server.close()

    def best_at(rows):
        ok = [r for r in rows if r["p99_ms"] <= p99_target_ms]
        return max((r["throughput_req_s"] for r in ok), default=0.0)

    return {
        "workload": "requests drawn per family uniformly from {16x16 3->8 n=512}, {32x32 64->64 n=1024 pixel, "
                    "hidden}, {the 7 stack layers}, {64x64(56) 64->64, 128x128 3->64 7x7}; one image each, "
                    "fresh inputs; open-loop Poisson arrivals",
        "budget_gb": budget_gb,
        "nstreams": nstreams,
        "max_batch": max_batch,
        "requests_per_rate": n_req,
        "latency": "scheduled arrival to completion (server clock)",
        "sweep": batched,
        "seeded_sweep": seeded,
        "sequential_sweep": sequential,
        "p99_target_ms": p99_target_ms,
        "served_req_s_at_p99_target": {"continuous_batching": best_at(batched),
                                       "sequential": best_at(sequential),
                                       "seeded": best_at(seeded) if seeded else None},
        "peak_budget_used_gb": st["peak_used_bytes"] / (1 << 30),
        "batches": st["batches"],
        "bit_exact": all(r["bit_exact"] for r in batched + seeded + sequential),
    }


# the paper's Table 4 convolution benchmarks: input H x W x Cin, filters kh x kw x Cout
PACKED_WORKLOADS = {
    "table4_32x32x32_3x3x32": dict(H=32, W=32, ih=32, Cin=32, Cout=32, k=3),
    "table4_28x28x1_5x5x5": dict(H=32, W=32, ih=28, Cin=1, Cout=5, k=5),
}
# a radix-2 butterfly of the packed transforms: three 32-bit multiplies at a
# quarter of the vector rate (12 issue slots) and about six full-rate ops
PACKED_SLOTS_PER_BUTTERFLY = 18


def packed_step(name: str, pset: str, B: int, steps: int, warmup: int, seed: int, rerandomize: bool = True):
    """The packed (BFV) secure convolution of one of Table 4's benchmarks on
    B images under one of Table 2's parameter sets: per step the client's
    NTT2D and Enc, the server's masks, HomConv and (for circuit privacy)
    re-randomisation, the client's Dec, fold and INTT2D, and the server's
    share; the filters are prepared once (setup). Every kernel timed with HIP
    events; the result checked against the cyclic convolution mod t."""
    import numpy as np
    import torch

    from types import SimpleNamespace

    from paper_2003_05328_amd import configs
    from paper_2003_05328_amd.ensei import Context
    from paper_2003_05328_amd.ensei_bfv import BfvContext, geometry

    pr = SimpleNamespace(**configs.PACKED_SETS[pset])
    pr.delta = (pr.q0 * pr.q1 + pr.t // 2) // pr.t
    wl = PACKED_WORKLOADS[name]
    H, W, Cin, Cout, k = wl["H"], wl["W"], wl["Cin"], wl["Cout"], wl["k"]
    F, n = H * W, pr.n
    P, K, G = geometry(Cin, F, n)
    g = np.random.default_rng(seed)
    dv = "cuda:0"
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dv)
    x = np.zeros((B, Cin, H, W), dtype=np.uint32)
    x[:, :, :wl["ih"], :wl["ih"]] = g.integers(0, 256, size=(B, Cin, wl["ih"], wl["ih"]))
    w = g.integers(-8, 9, size=(Cout, Cin, k, k)).astype(np.int32)
    s = g.integers(-1, 2, size=n).astype(np.int8)
    e = np.rint(g.normal(0, 4.0, size=(B * G * K, n))).astype(np.int32)
    e_pk = np.rint(g.normal(0, 4.0, size=(1, n))).astype(np.int32)
    r = g.integers(0, pr.t, size=(B * Cout * K, n)).astype(np.uint32)
    c = BfvContext(pr.t, pr.q0, pr.q1, n, 0)
    lwe = Context(pr.t, 0)
    xd, sd, ed, rd = d(x), d(s), d(e), d(r)
    # setup: the client's key and public key, the server's filters
    s_hat = c.key(sd)
    pk = c.encrypt(torch.zeros((1, 1, n), dtype=torch.uint32, device=dv), s_hat, d(e_pk), seed ^ 0x9E37)
    w_enc = c.encode_filters(lwe.weight_prep(d(w), H, W))
    x_hat = torch.empty((B, Cin, F), dtype=torch.uint32, device=dv)
    ct_in = torch.empty((B * G * K, 2, 2, n), dtype=torch.uint32, device=dv)
    mask = torch.empty((B * Cout * K, 2, n), dtype=torch.uint32, device=dv)
    ct_out = torch.empty((B * Cout * K, 2, 2, n), dtype=torch.uint32, device=dv)
    v = torch.empty((B * Cout * K, n), dtype=torch.uint32, device=dv)
    y = torch.empty((B, Cout, F), dtype=torch.uint32, device=dv)
    s_a = torch.empty((B * Cout, F), dtype=torch.uint32, device=dv)
    rf = torch.empty((B, Cout, F), dtype=torch.uint32, device=dv)
    s_b = torch.empty((B * Cout, F), dtype=torch.uint32, device=dv)
    flood = min(pr.delta // 16, 2**30)
    names = ["ntt2d", "encrypt", "encode_masks", "homconv", "rerandomize", "decrypt", "fold", "intt2d",
             "server_share"]

    def step(ev=None):
        mark = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
        mark(0)
        lwe.ntt2d(xd, out=x_hat)
        mark(1)
        c.encrypt(x_hat, s_hat, ed, seed, out=ct_in)
        mark(2)
        c.encode_masks(rd, out=mask)
        mark(3)
        c.homconv(ct_in, w_enc, mask, B, Cin, F, out=ct_out)
        mark(4)
        if rerandomize:
            c.rerandomize(ct_out, pk[0], seed ^ 0x5EED, flood)
        mark(5)
        c.decrypt(ct_out, s_hat, out=v)
        mark(6)
        c.fold(v, B, Cout, F, out=y)
        mark(7)
        lwe.intt2d(y.view(B * Cout, F), H, W, out=s_a)
        mark(8)
        c.fold(rd, B, Cout, F, negate=True, out=rf)
        lwe.intt2d(rf.view(B * Cout, F), H, W, out=s_b)
        mark(9)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    for ev in events:
        step(ev)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    us = {nm: float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in events])) * 1e3 for i, nm in enumerate(names)}
    # check: the shares add up to the cyclic convolution mod t (direct loops at sampled positions)
    y_sh = (s_a.cpu().numpy().astype(np.int64) + s_b.cpu().numpy()).reshape(B, Cout, H, W) % pr.t
    ok = True
    for _ in range(16):
        b, o, m1, m2 = (int(g.integers(B)), int(g.integers(Cout)), int(g.integers(H)), int(g.integers(W)))
        acc = sum(int(w[o, i, j1, j2]) * int(x[b, i, (m1 - j1) % H, (m2 - j2) % W])
                  for i in range(Cin) for j1 in range(k) for j2 in range(k))
        ok &= acc % pr.t == int(y_sh[b, o, m1, m2])
    # butterflies of each transform-bearing kernel per step
    bf = (n // 2) * (n.bit_length() - 1)
    nin, nout = B * G * K, B * Cout * K
    transforms = {"encrypt": 3 * nin, "encode_masks": 3 * nout, "rerandomize": 6 * nout if rerandomize else 0,
                  "decrypt": 3 * nout}
    dom = max(transforms, key=lambda kk: us[kk])
    peak = 256 * 64 * 2.4e9 / PACKED_SLOTS_PER_BUTTERFLY
    ach = transforms[dom] * bf / (us[dom] * 1e-6)
    c.close()
    lwe.close()
    return {"workload": f"{name} (paper Table 4), batch {B}, Table 2 set {pset}: t={pr.t}, q={pr.q0}*{pr.q1}, "
                        f"n={n}, {G * K} input and {Cout * K} output ciphertexts per image",
            "images_per_s": B / (ms * 1e-3), "ms_per_step": ms, "kernels_us": us, "rerandomized": rerandomize,
            "roofline": {"kernel": dom, "bound": "alu", "achieved": ach, "peak": peak, "unit": "butterfly/s",
                         "frac": ach / peak, "butterflies": transforms[dom] * bf,
                         "peak_derivation": "256 CUs x 64 lanes x 2.4 GHz / 18 issue slots per butterfly"},
            "verified": bool(ok)}


def host_cpu():
    """The host's CPU model and usable cores (os.sched_getaffinity)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def oracle_stage_ms(orc, inp, reps: int = 3):
    """The oracle's whole step of one layer, each stage timed on its own:
    median of `reps` per stage, milliseconds."""
    import numpy as np

    S, P = inp.shape, inp.p
    st = {}

    def t(name, fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            ts.append((time.perf_counter() - t0) * 1e3)
        st[name] = float(np.median(ts))
        return out

    x_hat = t("ntt2d", lambda: orc.ntt2d(inp.x, P)).reshape(S.B, S.Cin, S.F)
    w_hat = t("weight_prep", lambda: orc.weight_prep(inp.w, S.H, S.W, P))
    ct_in = t("encrypt", lambda: orc.encrypt(x_hat, inp.s, inp.e, inp.seed_a, P))
    ct_out = t("homconv", lambda: orc.homconv(ct_in, w_hat, inp.r, P))
    del ct_in
    m = t("decrypt", lambda: orc.decrypt(ct_out, inp.s, P))
    del ct_out
    t("intt2d", lambda: orc.ntt2d(m.reshape(S.B, S.Cout, S.H, S.W), P, inverse=True))
    t("server_share", lambda: orc.server_share(inp.r, S.H, S.W, P))
    return st


def cpu_baseline(shapes, seed: int, threads: int, single_layer: int | None, setup_in_step: bool = False):
    """The CPU oracle (plain C, gcc -O2, OpenMP) on the host: one image of
    every layer in `shapes`, each stage the median of three runs, on
    `threads` threads; and one image of layer `single_layer` single-threaded
    (None: skip). The filters' preparation counts in the step only with
    setup_in_step (as in the GPU step it is compared with)."""
    import dataclasses

    import oracle
    from paper_2003_05328_amd import configs, synth

    orc = oracle.default()
    model, ncores = host_cpu()
    P = configs.P

    def layer_inputs(k, S):
        return synth.generate(dataclasses.replace(S, B=1), P, seed + 5000 + k)

    used = orc.set_threads(threads)
    per_layer, macs = [], 0
    for k, S in enumerate(shapes):
        st = oracle_stage_ms(orc, layer_inputs(k, S))
        per_layer.append(st)
        macs += S.Cout * S.Cin * S.F
    def step_ms(st):
        return sum(v for k, v in st.items() if setup_in_step or k != "weight_prep")

    total_ms = sum(step_ms(st) for st in per_layer)
    stages = {name: sum(st[name] for st in per_layer) for name in per_layer[0]}
    res = {"value": macs / (total_ms * 1e-3), "unit": "ct-MAC/s", "cores": used, "kind": "oracle",
           "sample": f"one image of each of the {len(shapes)} layers (the workload's per-image work), every stage "
                     f"(NTT2D, weight prep, Enc, HomConv, Dec, INTT2D, server share) timed as the median of 3 runs; "
                     f"weight prep {'in' if setup_in_step else 'outside'} the step, as on the GPU",
           "stages_ms": stages, "step_ms_per_image": total_ms, "nproc": ncores, "cpu_model": model}
    if single_layer is not None:
        orc.set_threads(1)
        S = shapes[single_layer]
        st = oracle_stage_ms(orc, layer_inputs(single_layer, S))
        ms = step_ms(st)
        res["single_thread"] = {"value": S.Cout * S.Cin * S.F / (ms * 1e-3), "unit": "ct-MAC/s", "cores": 1,
                                "sample": f"one image of layer {single_layer + 1} ({S.H}x{S.W}, {S.Cin}->{S.Cout}), "
                                          f"each stage the median of 3 runs", "stages_ms": st, "step_ms": ms}
        orc.set_threads(used)
    return res


def stack_layers(ctx, seed: int, seeded: bool = False, shapes=None):
    """Inputs and output buffers of the stack's layers for a plan."""
    import numpy as np
    import torch

    from paper_2003_05328_amd import configs, synth
    from paper_2003_05328_amd.ensei import Plan

    shapes = shapes or configs.stack_shapes(B=8)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    inps, layers = [], []
    for i, S in enumerate(shapes):
        inp = synth.generate(S, configs.P, seed + 1000 + i)
        l = {"H": S.H, "W": S.W, "Cin": S.Cin, "Cout": S.Cout, "kh": S.kh, "kw": S.kw, "n": S.n,
             "seed_a": inp.seed_a, "w": d(inp.w), "x": d(inp.x), "s": d(inp.s), "e": d(inp.e), "r": d(inp.r)}
        l.update(Plan.buffers(ctx, S.H, S.W, S.Cin, S.Cout, S.n, S.B, seeded=seeded))
        inps.append(inp)
        layers.append(l)
    return shapes, inps, layers


def verify_layer(ctx, S, inp, l, samples: int = 8, seed: int = 0) -> bool:
    """Exact decryption (m = sum_i W^ x^ + r mod p, with W^ from the single
    weight-prep call) and the shares' sum at sampled positions against the
    cyclic convolution's definition, evaluated here by direct loops."""
    import numpy as np

    P = inp.p
    xh = l["x_hat"].cpu().numpy().astype(np.int64).reshape(S.B, S.Cin, S.F)
    wh = ctx.weight_prep(l["w"], S.H, S.W).cpu().numpy().astype(np.int64)
    m = l["m"].cpu().numpy().astype(np.int64).reshape(S.B, S.Cout, S.F)
    ok = bool(np.array_equal(m, (np.einsum("oif,bif->bof", wh, xh) + inp.r.reshape(S.B, S.Cout, S.F)) % P))
    y = (l["s_a"].cpu().numpy().astype(np.int64) + l["s_b"].cpu().numpy()).reshape(S.B, S.Cout, S.H, S.W) % P
    g = np.random.default_rng(seed)
    wmod = inp.w.astype(np.int64) % P
    for _ in range(samples):
        b, o, m1, m2 = (int(g.integers(S.B)), int(g.integers(S.Cout)), int(g.integers(S.H)), int(g.integers(S.W)))
        acc = 0
        for i in range(S.Cin):
            for j1 in range(S.kh):
                for j2 in range(S.kw):
                    acc += int(wmod[o, i, j1, j2]) * int(inp.x[b, i, (m1 - j1) % S.H, (m2 - j2) % S.W])
        ok &= (acc % P) == int(y[b, o, m1, m2])
    return ok


STAGES = ("client_ntt2d_enc", "server_homconv", "dec_intt2d_share")


def stack_main(ctx, args):
    """The headline: the seven-layer stack (batch 8) as a batched plan, one
    plan run per step, each stage timed with HIP events on its stream."""
    import numpy as np
    import torch

    from paper_2003_05328_amd.ensei import Plan, lib

    shapes, inps, layers = stack_layers(ctx, args.seed)
    t0 = time.perf_counter()
    plan = Plan(ctx, layers)
    create_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    verified = all(verify_layer(ctx, S, inp, l, seed=i) for i, (S, inp, l) in enumerate(zip(shapes, inps, layers)))
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ev in events:
        ev[0].record()
        for k in range(3):
            plan.run_stage(k)
            ev[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    stage_us = {nm: float(np.mean([ev[k].elapsed_time(ev[k + 1]) for ev in events])) * 1e3
                for k, nm in enumerate(STAGES)}
    hc_us = stage_us["server_homconv"]
    macs = sum(S.B * S.Cout * S.Cin * S.F for S in shapes)
    per_layer = []
    for S in shapes:
        nbytes = homconv_bytes(S, int(lib().ensei_wpack_bytes(S.Cout, S.Cin, S.F)))
        i8 = 21 * S.B * S.Cout * S.Cin * S.F * (S.n + 1)
        per_layer.append({"layer": f"{S.H}x{S.W} {S.Cin}->{S.Cout}", "algorithmic_bytes": nbytes, "i8_macs": i8,
                          "bound_us": max(nbytes / (HBM_PEAK_GBS * 1e9), i8 / MFMA_I8_PEAK_MACS) * 1e6,
                          "bound": "hbm" if nbytes / (HBM_PEAK_GBS * 1e9) >= i8 / MFMA_I8_PEAK_MACS else "mfma"})
    hc_bytes = sum(r["algorithmic_bytes"] for r in per_layer)
    achieved = hc_bytes / (hc_us * 1e-6) / 1e9
    sched = plan.schedule()
    plan.close()
    return {
        "metric": "HomConv ciphertext-MACs/s (whole secure-conv step of the seven-layer stack, batch 8: NTT2D, "
                  "Enc, HomConv, Dec, INTT2D, server share; filters prepared once at plan creation)",
        "value": macs / (ms_per_step * 1e-3),
        "unit": "ct-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "stack8_7layers_3x3_n1024_b8",
            "layers": "(Cin,Cout,HxW) (3,64,32) (64,64,32) (64,128,16) (128,128,16) (128,256,8) (256,256,8) "
                      "(256,512,4)",
            "batch": 8, "lwe_n": 1024, "p": 65537, "q": "2^64", "ct_macs_per_step": macs,
            "schedule": sched, "plan_create_s": create_s,
        },
        "roofline": {
            "kernel": "HomConv stage of the plan (all seven layers' HomConv launches)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_entry(STACK_TRAFFIC_FILE),
            "algorithmic_bytes": hc_bytes,
            "avg_us": hc_us,
            "bound_us": sum(r["bound_us"] for r in per_layer),
            "frac_of_layer_bounds": sum(r["bound_us"] for r in per_layer) / hc_us,
            "per_layer": per_layer,
        },
        "stages_us": stage_us,
        "verified": bool(verified),
    }


def layer_main(ctx, S, inp, steps: int, warmup: int, homconv: str = "mfma", workload: str = None):
    """One layer's whole step through the single calls (filters prepared in
    every step), each kernel timed with HIP events on its stream."""
    import numpy as np
    import torch

    from paper_2003_05328_amd import configs
    from paper_2003_05328_amd.ensei import lib

    P = configs.P
    dv = "cuda:0"

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dv)

    x, w, s, e, r = d(inp.x), d(inp.w), d(inp.s), d(inp.e), d(inp.r)
    pack_bytes = int(lib().ensei_wpack_bytes(S.Cout, S.Cin, S.F))
    w_hat = torch.empty((S.Cout, S.Cin, S.F), dtype=torch.uint32, device=dv)
    pack = torch.empty((pack_bytes,), dtype=torch.int8, device=dv)
    x_hat = torch.empty((S.B, S.Cin, S.F), dtype=torch.uint32, device=dv)
    ct_in = torch.empty((S.B, S.F, S.n + 1, S.Cin), dtype=torch.uint64, device=dv)  # word-major
    ct_out = torch.empty((S.B, S.F, S.n + 1, S.Cout), dtype=torch.uint64, device=dv)
    m = torch.empty((S.B, S.Cout, S.F), dtype=torch.uint32, device=dv)
    s_a = torch.empty((S.B, S.Cout, S.H, S.W), dtype=torch.uint32, device=dv)
    s_b = torch.empty((S.B, S.Cout, S.H, S.W), dtype=torch.uint32, device=dv)
    torch.cuda.synchronize()
    names = ["weight_prep", "pack_weights", "ntt2d", "encrypt", "homconv", "decrypt", "intt2d", "server_share"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()

        mark(0)
        ctx.weight_prep(w, S.H, S.W, out=w_hat)
        mark(1)
        ctx.pack_weights(w_hat, out=pack)
        mark(2)
        ctx.ntt2d(x, out=x_hat)
        mark(3)
        ctx.encrypt(x_hat, s, e, inp.seed_a, out=ct_in)
        mark(4)
        if homconv == "mfma":
            ctx.homconv(ct_in, pack, r, S.Cout, out=ct_out)
        else:
            ctx.homconv_valu(ct_in, w_hat, r, out=ct_out)
        mark(5)
        ctx.decrypt(ct_out, s, out=m)
        mark(6)
        ctx.intt2d(m, S.H, S.W, out=s_a)
        mark(7)
        ctx.server_share(r, S.H, S.W, out=s_b)
        mark(8)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    l = {"x_hat": x_hat, "w": w, "m": m, "s_a": s_a, "s_b": s_b}
    ok = verify_layer(ctx, S, inp, l, samples=32)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    per_kernel_ms = {nm: float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in events])) for i, nm in enumerate(names)}
    hc_ms = per_kernel_ms["homconv"]
    macs = S.B * S.Cout * S.Cin * S.F
    hc_bytes = homconv_bytes(S, pack_bytes)
    achieved = hc_bytes / (hc_ms * 1e-3) / 1e9
    kname = homconv_kernel_name(S) if homconv == "mfma" else "homconv_valu_kernel"
    return {
        "value": macs / (ms_per_step * 1e-3),
        "unit": "ct-MAC/s",
        "ms_per_step": ms_per_step,
        "config": {"workload": None, "grid": f"{S.H}x{S.W}", "cin": S.Cin, "cout": S.Cout, "kernel": f"{S.kh}x{S.kw}",
                   "lwe_n": S.n, "batch": S.B, "p": P, "q": "2^64", "homconv": homconv},
        "roofline": {
            "kernel": kname,
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_entry(workload=workload, kernel=kname) if homconv == "mfma" else None,
            "algorithmic_bytes": hc_bytes, "avg_us": hc_ms * 1e3,
        },
        "kernels_us": {k: v * 1e3 for k, v in per_kernel_ms.items()},
        "word_mac_per_s_homconv": macs * (S.n + 1) / (hc_ms * 1e-3),
        "verified": ok,
    }


def cpu_threads(args) -> int:
    if args.cpu_threads > 0:
        return args.cpu_threads
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else len(os.sched_getaffinity(0))


def main():
    args = parse()
    if args.probe_copy:
        probe_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported "
                          "(HomConv shards over frequencies with no exchange, see the design notes)"}))
        sys.exit(2)
    from paper_2003_05328_amd import configs, synth
    from paper_2003_05328_amd.ensei import Context

    ctx = Context(configs.P, 0)
    if args.seeded:
        S = configs.WORKLOADS[LAYER_WORKLOAD if args.workload == DEFAULT_WORKLOAD else args.workload]
        res = seeded_step(ctx, S, synth.generate(S, configs.P, args.seed), args.steps, args.warmup)
        print(json.dumps({"metric": "HomConv ciphertext-MACs/s, whole secure-conv step with seeded ciphertexts",
                          "value": res["ct_mac_per_s"], "unit": "ct-MAC/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
                          "config": {"workload": LAYER_WORKLOAD}, "seeded": res}), flush=True)
        sys.exit(0 if res["verified"] else 3)
    if args.ntt:
        stack = configs.stack_shapes(B=8)
        big = configs.WORKLOADS["conv64x64(56)_c64to64_k3_n1024"]
        res = {"stack8_weight_prep": ntt_throughput(ctx, [(S.Cout * S.Cin, S.H, S.W) for S in stack]),
               "conv64x64_weight_prep": ntt_throughput(ctx, [(big.Cout * big.Cin, big.H, big.W)])}
        main_row = res["conv64x64_weight_prep"]
        print(json.dumps({"metric": "NTT2D points/s (64x64 weight batch, caches flushed before each launch)",
                          "value": main_row["points_per_s"], "unit": "points/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "u32", "data": "synthetic",
                          "config": {"workload": "conv64x64_weight_prep"}, "ntt2d": res}), flush=True)
        return
    if args.chained:
        res = chained(ctx, args.steps, args.seed)
        print(json.dumps({"metric": "chained secure-conv rounds: ciphertext-MACs/s over both rounds",
                          "value": res["ct_mac_per_s"], "unit": "ct-MAC/s", "n_gpus": 1, "steps": args.steps,
                          "higher_is_better": True, "dtype": "u64", "data": "synthetic",
                          "config": {"workload": res["workload"]}, "chained": res}), flush=True)
        sys.exit(0 if res["bit_exact"] else 3)
    if args.packed:
        rows = [packed_step(nm, ps, args.packed_batch, args.steps, args.warmup, args.seed)
                for nm in PACKED_WORKLOADS for ps in ("binary", "high")]
        main_row = rows[0]
        print(json.dumps({"metric": "packed (BFV) secure convolutions: images/s", "value": main_row["images_per_s"],
                          "unit": "images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "higher_is_better": True, "dtype": "u32", "data": "synthetic",
                          "config": {"workload": main_row["workload"]}, "roofline": main_row["roofline"],
                          "packed": rows}), flush=True)
        sys.exit(0 if all(r["verified"] for r in rows) else 3)
    if args.serve:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        res = serving(ctx, rates, args.serve_requests, args.serve_budget_gb, args.seed, nstreams=args.serve_streams,
                      max_batch=args.serve_max_batch, seeded_rates=rates[-2:])
        at = res["served_req_s_at_p99_target"]["continuous_batching"]
        print(json.dumps({"metric": f"served secure-conv requests/s at p99 <= {res['p99_target_ms']:.0f} ms "
                                    "(mixed shapes, continuous batching)",
                          "value": at, "unit": "req/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64",
                          "data": "synthetic", "config": {"workload": "serving"}, "serving": res}), flush=True)
        sys.exit(0 if res["bit_exact"] else 3)

    if args.workload != DEFAULT_WORKLOAD:
        # one layer's step through the single calls
        S = configs.WORKLOADS[args.workload]
        inp = synth.generate(S, configs.P, args.seed)
        res = layer_main(ctx, S, inp, args.steps, args.warmup, args.homconv, workload=args.workload)
        res["config"]["workload"] = args.workload
        result = {"metric": "HomConv ciphertext-MACs/s (whole secure-conv step of one layer: NTT2D, weight prep, "
                            "Enc, HomConv, Dec, INTT2D, server share)",
                  "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1, "steps": args.steps,
                  "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"), "higher_is_better": True,
                  "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic"}
        result.update(res)
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = cpu_baseline([S], args.seed, cpu_threads(args), 0, setup_in_step=True)
        print(json.dumps(result), flush=True)
        sys.exit(0 if result["verified"] else 3)

    import torch

    result = stack_main(ctx, args)
    torch.cuda.empty_cache()
    if not args.no_extras:
        S = configs.WORKLOADS[LAYER_WORKLOAD]
        inp = synth.generate(S, configs.P, args.seed)
        layer = layer_main(ctx, S, inp, max(args.steps, 20), max(args.warmup, 10), workload=LAYER_WORKLOAD)
        layer["config"]["workload"] = LAYER_WORKLOAD
        result["layer_conv32x32"] = layer
        result["verified"] = result["verified"] and layer["verified"]
        torch.cuda.empty_cache()
        stack = configs.stack_shapes(B=8)
        big = configs.WORKLOADS["conv64x64(56)_c64to64_k3_n1024"]
        result["ntt2d"] = {
            "stack8_weight_prep": ntt_throughput(ctx, [(S.Cout * S.Cin, S.H, S.W) for S in stack]),
            "conv64x64_weight_prep": ntt_throughput(ctx, [(big.Cout * big.Cin, big.H, big.W)]),
        }
        result["seeded"] = seeded_step(ctx, S, inp, max(args.steps, 20), max(args.warmup, 10))
        result["verified"] = result["verified"] and result["seeded"]["verified"]
        torch.cuda.empty_cache()
        result["homconv_layers"] = homconv_layers(ctx)
        result["batched"] = stack_batched(ctx, args.stack_reps, args.seed)
        result["verified"] = (result["verified"] and result["batched"]["bit_exact_vs_sequential"]
                              and result["batched"]["seeded"]["bit_exact_vs_unseeded"])
        torch.cuda.empty_cache()
        result["chained"] = chained(ctx, args.stack_reps, args.seed)
        result["verified"] = result["verified"] and result["chained"]["bit_exact"]
        torch.cuda.empty_cache()
        result["packed"] = [packed_step("table4_32x32x32_3x3x32", ps, args.packed_batch, max(args.steps, 10),
                                        max(args.warmup, 3), args.seed) for ps in ("binary", "high")]
        result["verified"] = result["verified"] and all(r["verified"] for r in result["packed"])
        torch.cuda.empty_cache()
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        result["serving"] = serving(ctx, rates, args.serve_requests, args.serve_budget_gb, args.seed,
                                    nstreams=args.serve_streams, max_batch=args.serve_max_batch,
                                    seeded_rates=rates[-2:])
        result["verified"] = result["verified"] and result["serving"]["bit_exact"]
    if not args.no_cpu_baseline:
        # all threads on one image of every stack layer; single-threaded on one image of the last layer
        result["cpu_baseline"] = cpu_baseline(configs.stack_shapes(B=8), args.seed, cpu_threads(args), 6)
    print(json.dumps(result), flush=True)
    if not result["verified"]:
        sys.exit(3)


if __name__ == "__main__":
    main()
