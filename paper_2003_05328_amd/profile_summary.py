"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2003_05328_amd.profile_summary --workload NAME \
        --trace DIR [--fetch DIR --write DIR --copy-fetch DIR --copy-write DIR] \
        --command "..." [--command "..."] --out profiles/NAME.md [--traffic profiles/homconv_traffic.json]

DIR is a rocprofv3 output directory written with `-o run --output-format csv`
(run_kernel_stats.csv for --kernel-trace --stats, run_counter_collection.csv
for --pmc). The HBM counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are
calibrated against a plain copy kernel of known size (the torch elementwise
kernel of `bench.py --probe-copy`, which reads and writes 1 GiB): the factor
is true bytes / counted bytes, applied per direction.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
HOMCONV_SRC = os.path.join(HERE, "csrc", "homconv.hip")


def code_digest(path: str) -> str:
    """SHA-256 of a source file's code: // comments and blank lines removed,
    so that counters stay attached to a kernel across edits of its comments
    only (the sources hold no string literal containing //)."""
    lines = []
    for line in open(path, encoding="utf-8"):
        code = line.split("//", 1)[0].rstrip()
        if code:
            lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()
COPY_BYTES = 1 << 30  # bench.py --probe-copy: 1 GiB read, 1 GiB written per launch


def short_name(kernel: str) -> str:
    name = kernel.split("(")[0]
    name = re.sub(r"^void ", "", name)
    return name.replace("ensei::", "")


def kernel_stats(trace_dir: str):
    rows = []
    with open(os.path.join(trace_dir, "run_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                         float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return rows


def counter_means(pmc_dir: str, counter: str):
    """Mean counter value per kernel (short name) over its dispatches."""
    acc = defaultdict(list)
    with open(os.path.join(pmc_dir, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def stage_runs(pmc_dir: str, counter: str, prefix: str):
    """The dispatches of kernels whose short name starts with prefix, in
    dispatch order, grouped into runs of consecutive such dispatches (one
    run per step's stage: the stages are separated by other kernels, and the
    number of launches in a stage may differ between runs of the plan's
    tuner). Each run is a list of (kernel, counter KiB)."""
    rows = []
    with open(os.path.join(pmc_dir, "run_counter_collection.csv")) as fh:
        for i, r in enumerate(csv.DictReader(fh)):
            if r["Counter_Name"] == counter:
                rows.append((int(r.get("Dispatch_Id") or i), short_name(r["Kernel_Name"]), float(r["Counter_Value"])))
    rows.sort()
    runs, cur = [], []
    for _, k, v in rows:
        if k.startswith(prefix):
            cur.append((k, v))
        elif cur:
            runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    return runs


def stage_kib(pmc_dir: str, counter: str, prefix: str, steps: int):
    """Counter KiB of one step's stage (mean over the last `steps` runs of
    stage_runs) and the last run's dispatches."""
    runs = stage_runs(pmc_dir, counter, prefix)
    assert len(runs) >= steps, "fewer stage runs than requested"
    last = runs[-steps:]
    return sum(sum(v for _, v in r) for r in last) / steps, last[-1]


def step_kernels(trace_dir: str, per_step: int, steps: int):
    """The last steps * per_step dispatches of run_kernel_trace.csv (start
    order): per kernel, calls per step and mean microseconds per call, and the
    order of one step's kernels."""
    rows = []
    with open(os.path.join(trace_dir, "run_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"])))
    rows.sort()
    last = rows[-per_step * steps:]
    agg = defaultdict(list)
    for a, b, k in last:
        agg[k].append((b - a) / 1e3)
    order = [k for _, _, k in last[-per_step:]]
    return {k: (len(v) / steps, sum(v) / len(v)) for k, v in agg.items()}, order


def copy_factor(pmc_dir: str, counter: str) -> float:
    """True bytes / counted bytes for the copy kernel (largest mean among its dispatches)."""
    means = counter_means(pmc_dir, counter)
    kib = max(v for k, v in means.items() if "elementwise" in k)
    return COPY_BYTES / (kib * 1024.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--kernel", default="homconv_mfma_kernel", help="kernel whose HBM bytes are recorded")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic")
    ap.add_argument("--stage-prefix", help="sum the HBM bytes of one step's dispatches of these kernels")
    ap.add_argument("--per-step", type=int, default=0, help="dispatches of one step in the trace")
    ap.add_argument("--steps", type=int, default=1, help="trace steps whose dispatches are averaged (the last ones)")
    ap.add_argument("--pmc-steps", type=int, default=1, help="counter-run steps averaged (the last ones)")
    ap.add_argument("--sq", action="append", default=[],
                    help="a --pmc run directory whose counters are listed per kernel (mean per dispatch)")
    ap.add_argument("--sq-prefix", default="", help="only kernels whose short name starts with this")
    args = ap.parse_args()

    lines = [f"# Kernel times and HBM traffic: {args.workload}", ""]
    lines.append("Commands (run from the repository root on one MI355X; OUT is any output directory):")
    lines.append("")
    for c in args.command:
        lines.append(f"    {c}")
    lines += ["", "## rocprofv3 --kernel-trace --stats", "",
              "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for name, calls, avg, mn, mx, pct in kernel_stats(args.trace):
        lines.append(f"| {name} | {calls} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {pct:.1f} |")

    if args.per_step:
        per, order = step_kernels(args.trace, args.per_step, args.steps)
        lines += ["", f"## One step ({args.per_step} dispatches; the last {args.steps} steps of the trace)", "",
                  "| kernel | calls per step | avg us | us per step |", "|---|---|---|---|"]
        tot = 0.0
        for k, (calls, avg) in sorted(per.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            lines.append(f"| {k} | {calls:g} | {avg:.1f} | {calls * avg:.1f} |")
            tot += calls * avg
        if args.stage_prefix:
            st = sum(c * a for k, (c, a) in per.items() if k.startswith(args.stage_prefix))
            lines += ["", f"Kernel time per step: {tot:.1f} us, of which {args.stage_prefix}* {st:.1f} us."]
        lines += ["", "One step's dispatch order: " + ", ".join(order)]

    record = None
    if args.fetch and args.write and args.copy_fetch and args.copy_write and not args.stage_prefix:
        ff, fw = copy_factor(args.copy_fetch, "FETCH_SIZE"), copy_factor(args.copy_write, "WRITE_SIZE")
        fetch, write = counter_means(args.fetch, "FETCH_SIZE"), counter_means(args.write, "WRITE_SIZE")
        lines += ["", "## HBM counters (rocprofv3 --pmc, one counter per run)", "",
                  f"Copy-kernel calibration (1 GiB each way): FETCH_SIZE x {ff:.3f}, WRITE_SIZE x {fw:.3f}.", "",
                  "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch (calibrated) |", "|---|---|---|---|"]
        for name in sorted(set(fetch) | set(write)):
            if "elementwise" in name or "copyBuffer" in name:
                continue
            fk, wk = fetch.get(name, 0.0), write.get(name, 0.0)
            hbm = fk * 1024 * ff + wk * 1024 * fw
            lines.append(f"| {name} | {fk:.0f} | {wk:.0f} | {hbm / 1e6:.1f} MB |")
            if args.kernel in name and record is None:
                record = {
                    "kernel": name,
                    "workload": args.workload,
                    "hbm_bytes_per_launch": int(round(hbm)),
                    "fetch_kib": fk,
                    "write_kib": wk,
                    "fetch_factor": ff,
                    "write_factor": fw,
                    "code_sha256": code_digest(HOMCONV_SRC),
                }
    if args.stage_prefix and args.fetch and args.write and args.copy_fetch and args.copy_write:
        ff, fw = copy_factor(args.copy_fetch, "FETCH_SIZE"), copy_factor(args.copy_write, "WRITE_SIZE")
        fk, flast = stage_kib(args.fetch, "FETCH_SIZE", args.stage_prefix, args.pmc_steps)
        wk, wlast = stage_kib(args.write, "WRITE_SIZE", args.stage_prefix, args.pmc_steps)
        hbm = fk * 1024 * ff + wk * 1024 * fw
        lines += ["", f"## One step's {args.stage_prefix}* dispatches (mean of the last {args.pmc_steps} steps of the "
                      "counter runs)", "",
                  f"FETCH_SIZE {fk:.0f} KiB, WRITE_SIZE {wk:.0f} KiB: {hbm / 1e6:.1f} MB of HBM traffic per step "
                  "(calibrated)."]
        if [k for k, _ in flast] == [k for k, _ in wlast]:
            lines += ["", "The last step's dispatches (calibrated MB):", "",
                      "| dispatch | kernel | fetched | written |", "|---|---|---|---|"]
            for i, ((k, fv), (_, wv)) in enumerate(zip(flast, wlast)):
                lines.append(f"| {i + 1} | {k} | {fv * 1024 * ff / 1e6:.1f} | {wv * 1024 * fw / 1e6:.1f} |")
        else:
            # the two counter runs' plans chose different launches (the
            # tuner times its candidates in each run): each run's own list
            for title, last, factor in (("fetched, FETCH_SIZE run", flast, ff), ("written, WRITE_SIZE run", wlast, fw)):
                lines += ["", f"The last step's dispatches, {title} (calibrated MB):", "",
                          "| dispatch | kernel | MB |", "|---|---|---|"]
                for i, (k, v) in enumerate(last):
                    lines.append(f"| {i + 1} | {k} | {v * 1024 * factor / 1e6:.1f} |")
        record = {"kernel": f"{args.stage_prefix}* (one step)", "workload": args.workload,
                  "hbm_bytes_per_launch": int(round(hbm)), "fetch_kib": fk, "write_kib": wk, "fetch_factor": ff,
                  "write_factor": fw, "code_sha256": code_digest(HOMCONV_SRC)}
    for sq_dir in args.sq:
        per = defaultdict(lambda: defaultdict(list))
        with open(os.path.join(sq_dir, "run_counter_collection.csv")) as fh:
            disp = defaultdict(lambda: defaultdict(float))
            names = {}
            for r in csv.DictReader(fh):
                k = short_name(r["Kernel_Name"])
                if not k.startswith(args.sq_prefix):
                    continue
                d = int(r["Dispatch_Id"])
                names[d] = k
                disp[d][r["Counter_Name"]] += float(r["Counter_Value"])
        for d, cs in disp.items():
            for c, v in cs.items():
                per[names[d]][c].append(v)
        counters = sorted({c for cs in per.values() for c in cs})
        lines += ["", f"## Counters of `{os.path.basename(os.path.normpath(sq_dir))}` (mean per dispatch, summed "
                      "over the device's instances)", "",
                  "| kernel | dispatches | " + " | ".join(counters) + " |",
                  "|---|---|" + "---|" * len(counters)]
        for k in sorted(per):
            n = max(len(v) for v in per[k].values())
            vals = [sum(per[k][c]) / len(per[k][c]) if per[k].get(c) else 0.0 for c in counters]
            lines.append(f"| {k} | {n} | " + " | ".join(f"{v:.0f}" for v in vals) + " |")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if args.traffic and record is not None:
        with open(args.traffic, "w") as fh:
            json.dump(record, fh, indent=1)
            fh.write("\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
