"""Short text summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2406_03466_amd.profile_summary stats DIR/run_kernel_stats.csv OUT.md --command "..." --title "..."
    python -m paper_2406_03466_amd.profile_summary hbm --kernel k_rtile_adj --name rtile_adj --workload qcl20_L8 \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv --out-dir profiles --command "..."
    python -m paper_2406_03466_amd.profile_summary counters C.csv OUT.md --command "..." --title "..."
    python -m paper_2406_03466_amd.profile_summary trace T.csv OUT.md --kernel NAME --last N --command "..." --title "..."
    python -m paper_2406_03466_amd.profile_summary mfma C.csv AGENT.csv OUT.md --kernel NAME --last N --command "..." --title "..."

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
    for f in ["kernels.hip", "engine.h", "tile_device.h", "jit.cpp"]:
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


def _per_kernel(path, counter, needle, last=0):
    """Counter values of the dispatches whose kernel name holds `needle`, in dispatch order; with `last`,
    only the last that many (the timed step's launches, after any tuning or warm-up launches)."""
    vals = []
    for r in sorted(_rows(path), key=lambda r: int(r["Dispatch_Id"])):
        if r["Counter_Name"] == counter and needle in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    return vals[-last:] if last else vals


def trace(args):
    """Average duration of the last N dispatches of a kernel from a rocprofv3 kernel trace."""
    rows = [r for r in _rows(args.csv) if args.kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    rows = rows[-args.last:]
    ms = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in rows]
    avg = sum(ms) / len(ms)
    out = [f"# {args.title}", "", "Command (from the repository root on the MI355X box):", "", "```", args.command,
           "```", "", f"* kernel: `{args.kernel}`; the last {len(ms)} dispatches (the timed steps)",
           f"* average duration: {avg:.4f} ms (min {min(ms):.4f}, max {max(ms):.4f})",
           "* per dispatch (ms): " + ", ".join(f"{m:.4f}" for m in ms)]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")


def mfma(args):
    """MFMA use of the last N dispatches of a kernel, from a counter run with SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_INSTS_MFMA and GRBM_GUI_ACTIVE. GRBM_GUI_ACTIVE is summed over the XCDs, so the wall-clock cycles of
    a dispatch are GRBM_GUI_ACTIVE / XCDs and its SIMD-cycles that many times the SIMD count; the busy
    fraction is SQ_VALU_MFMA_BUSY_CYCLES over those SIMD-cycles."""
    agent = [r for r in _rows(args.agent) if r["Agent_Type"] == "GPU"][0]
    xcc, simds = int(agent["Num_Xcc"]), int(agent["Simd_Count"])
    per = defaultdict(dict)
    for r in _rows(args.csv):
        if args.kernel in r["Kernel_Name"]:
            i = int(r["Dispatch_Id"])
            per[i][r["Counter_Name"]] = float(r["Counter_Value"])
            per[i]["ms"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    ids = sorted(per)[-args.last:]
    out = [f"# {args.title}", "", "Command (from the repository root on the MI355X box):", "", "```", args.command,
           "```", "", f"* kernel: `{args.kernel}`, the last {len(ids)} dispatches; GPU: {xcc} XCDs, {simds} SIMDs",
           f"* flops per MFMA instruction: {args.flops_per_inst}",
           "* durations are those of the counter run (dispatches serialised by the profiler)", "",
           "| Dispatch | ms | MFMA instructions | TFLOP/s | MFMA busy fraction |", "|---:|---:|---:|---:|---:|"]
    tb = tc = tf = tm = 0.0
    for i in ids:
        v = per[i]
        cyc = v["GRBM_GUI_ACTIVE"] / xcc * simds
        fl = v["SQ_INSTS_MFMA"] * args.flops_per_inst
        tb += v["SQ_VALU_MFMA_BUSY_CYCLES"]; tc += cyc; tf += fl; tm += v["ms"]
        out.append(f"| {i} | {v['ms']:.2f} | {v['SQ_INSTS_MFMA']:.4g} | {fl / v['ms'] / 1e9:.1f} | "
                   f"{v['SQ_VALU_MFMA_BUSY_CYCLES'] / cyc:.3f} |")
    out.append(f"| all | {tm:.2f} | {tf / args.flops_per_inst:.4g} | {tf / tm / 1e9:.1f} | {tb / tc:.3f} |")
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")


def hbm(args):
    cf = _per_kernel(args.copy_fetch, "FETCH_SIZE", "copyBuffer")
    cw = _per_kernel(args.copy_write, "WRITE_SIZE", "copyBuffer")
    if not cf or not cw:
        raise SystemExit("no copy-kernel dispatches in the calibration files")
    fetch_factor = COPY_BYTES / (sum(cf) / len(cf) * 1024.0)
    write_factor = COPY_BYTES / (sum(cw) / len(cw) * 1024.0)
    f = _per_kernel(args.fetch, "FETCH_SIZE", args.kernel, args.last)
    w = _per_kernel(args.write, "WRITE_SIZE", args.kernel, args.last)
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
             f"* dispatches averaged: {len(f)}" + (f" (the last {args.last}: the timed step)" if args.last else ""),
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
    rows = [r for r in _rows(args.csv) if not args.needle or any(x in r["Kernel_Name"] for x in args.needle)]
    if args.last:  # per kernel, only its last `last` dispatches (the timed step)
        ids = defaultdict(set)
        for r in rows:
            ids[r["Kernel_Name"]].add(int(r["Dispatch_Id"]))
        keep = {k: set(sorted(v)[-args.last:]) for k, v in ids.items()}
        rows = [r for r in rows if int(r["Dispatch_Id"]) in keep[r["Kernel_Name"]]]
    for r in rows:
        name = r["Kernel_Name"]
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
    h.add_argument("--last", type=int, default=0, help="average only the last N dispatches of the kernel")
    h.set_defaults(fn=hbm)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--kernel", required=True)
    t.add_argument("--last", type=int, required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--title", required=True)
    t.set_defaults(fn=trace)
    m = sub.add_parser("mfma")
    m.add_argument("csv")
    m.add_argument("agent")
    m.add_argument("out")
    m.add_argument("--kernel", required=True)
    m.add_argument("--last", type=int, required=True)
    m.add_argument("--flops-per-inst", type=int, default=4096)
    m.add_argument("--command", required=True)
    m.add_argument("--title", required=True)
    m.set_defaults(fn=mfma)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--needle", action="append")
    c.add_argument("--last", type=int, default=0, help="per kernel, only its last N dispatches")
    c.set_defaults(fn=counters)
    args = ap.parse_args()
    args.fn(args)


if __name__ == "__main__":
    main()
