"""Short text summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2406_03466_amd.profile_summary stats DIR/run_kernel_stats.csv OUT.md --command "..." --title "..."
    python -m paper_2406_03466_amd.profile_summary hbm --kernel k_rtile_adj --name rtile_adj --workload qcl20_L8 \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv --out-dir profiles --command "..."
    python -m paper_2406_03466_amd.profile_summary counters C.csv OUT.md --command "..." --title "..."

`hbm` scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by what the same counters read for a plain
device copy of known size, averages them over the kernel's dispatches and writes
<name>_<workload>_pmc.json (read by bench.py while the kernel source is unchanged) plus a markdown note.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30   # bench.py --copy-calibration copies 2^27 doubles


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ["kernels.hip", "engine.h"]:
        with open(os.path.join(ROOT, "paper_2406_03466_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def stats(args):
    rows = _rows(args.csv)
    out = [f"# {args.title}", "", "Command (from the repository root on the MI355X box):", "", "```", args.command, "```", "",
           "| Kernel | Calls | Average (ms) | Min (ms) | Max (ms) | Total (ms) | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:args.top]:
        out.append(f"| `{r['Name'][:96]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                   f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")


def _per_kernel(path, counter, needle):
    vals = []
    for r in _rows(path):
        if r["Counter_Name"] == counter and needle in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    return vals


def hbm(args):
    cf = _per_kernel(args.copy_fetch, "FETCH_SIZE", "copyBuffer")
    cw = _per_kernel(args.copy_write, "WRITE_SIZE", "copyBuffer")
    if not cf or not cw:
        raise SystemExit("no copy-kernel dispatches in the calibration files")
    fetch_factor = COPY_BYTES / (sum(cf) / len(cf) * 1024.0)
    write_factor = COPY_BYTES / (sum(cw) / len(cw) * 1024.0)
    f = _per_kernel(args.fetch, "FETCH_SIZE", args.kernel)
    w = _per_kernel(args.write, "WRITE_SIZE", args.kernel)
    if not f or not w:
        raise SystemExit(f"no dispatches of {args.kernel}")
    fb = sum(f) / len(f) * 1024.0 * fetch_factor
    wb = sum(w) / len(w) * 1024.0 * write_factor
    d = {"kernel": args.kernel, "workload": args.workload, "dispatches": len(f),
         "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb,
         "fetch_calibration_factor": fetch_factor, "write_calibration_factor": write_factor,
         "kernel_source_hash": kernel_source_hash(), "command": args.command}
    if args.algorithmic_bytes:
        d["algorithmic_bytes_per_launch"] = args.algorithmic_bytes
        d["traffic_over_algorithmic"] = (fb + wb) / args.algorithmic_bytes
    base = os.path.join(args.out_dir, f"{args.name}_{args.workload}_pmc")
    with open(base + ".json", "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    lines = [f"# HBM traffic of `{args.kernel}` ({args.workload})", "", "Commands (from the repository root):", "",
             "```", args.command, "```", "",
             f"* dispatches averaged: {len(f)}",
             f"* calibration (plain 1 GiB device copy): FETCH_SIZE x {fetch_factor:.3f}, WRITE_SIZE x {write_factor:.3f}",
             f"* read per launch: {fb / 2**30:.4f} GiB; written per launch: {wb / 2**30:.4f} GiB; "
             f"total {(fb + wb) / 2**30:.4f} GiB"]
    if args.algorithmic_bytes:
        lines.append(f"* algorithmic bytes per launch: {args.algorithmic_bytes / 2**30:.4f} GiB "
                     f"(measured / algorithmic = {(fb + wb) / args.algorithmic_bytes:.3f})")
    lines.append(f"* kernel source hash: {d['kernel_source_hash']}")
    with open(base + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")


def counters(args):
    agg = defaultdict(float)
    n = defaultdict(int)
    for r in _rows(args.csv):
        name = r["Kernel_Name"]
        if args.needle and not any(x in name for x in args.needle):
            continue
        key = (name.split("(")[0][:60], r["Counter_Name"])
        agg[key] += float(r["Counter_Value"])
        n[key] += 1
    out = [f"# {args.title}", "", "Command (from the repository root on the MI355X box):", "", "```", args.command, "```", "",
           "| Kernel | Counter | Dispatches | Sum |", "|---|---|---:|---:|"]
    for (k, c), v in sorted(agg.items()):
        out.append(f"| `{k}` | {c} | {n[(k, c)]} | {v:.4g} |")
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--top", type=int, default=12)
    s.set_defaults(fn=stats)
    h = sub.add_parser("hbm")
    for k in ["--kernel", "--name", "--workload", "--fetch", "--write", "--copy-fetch", "--copy-write", "--out-dir",
              "--command"]:
        h.add_argument(k, required=True)
    h.add_argument("--algorithmic-bytes", type=int, default=0)
    h.set_defaults(fn=hbm)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--needle", action="append")
    c.set_defaults(fn=counters)
    args = ap.parse_args()
    args.fn(args)


if __name__ == "__main__":
    main()
