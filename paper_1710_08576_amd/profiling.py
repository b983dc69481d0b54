"""rocprofv3 summaries for the benchmark (kept as text under profiles/).

summarize() reads the CSV output of three rocprofv3 runs of bench.py -- a
kernel trace with --stats, a FETCH_SIZE pass and a WRITE_SIZE pass, each
with the HBM copy microbenchmark in the same process -- and writes a short
markdown summary with a machine-readable JSON block:

* per-kernel call counts and mean durations (trace);
* FETCH_SIZE / WRITE_SIZE per dispatch (KiB) for the filter kernels and the
  copy kernel;
* the calibration factors that make the copy kernel's counters equal its
  known traffic (one read and one write of the copied bytes);
* the calibrated HBM bytes per launch of each filter kernel;
* a hash of the kernel sources, so a later build can tell whether the
  counters still describe its kernels.

Usage:  python -m paper_1710_08576_amd.profiling --trace DIR --fetch DIR
        --write DIR --bench FILE --copy-bytes N --out profiles/NAME.md
        --command "..." [--command "..."]
        python -m paper_1710_08576_amd.profiling --trace DIR --trace-only
        --title "..." --out profiles/NAME.md --command "..."

The second form summarises a kernel trace alone: launches grouped by kernel
and grid size (the same kernel runs with different grids in different
workloads), with their mean durations.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/rfi_kernels.hip", "csrc/rfi_device.hpp", "csrc/rfi_internal.hpp",
                  "csrc/q8_table.inc"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _csv(directory, suffix):
    files = glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    rows = []
    for fn in files:
        with open(fn) as f:
            rows += list(csv.DictReader(f))
    return rows


def _counter_means(directory, counter):
    per = {}
    for r in _csv(directory, "_counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: statistics.mean(v) for k, v in per.items()}


def summarize(trace_dir, fetch_dir, write_dir, bench_file, copy_bytes, commands):
    stats = {}
    for r in _csv(trace_dir, "_kernel_stats.csv"):
        stats[r["Name"]] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                            "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "k_copy_tile" in k]
    if not copy:
        raise ValueError("no copy-kernel dispatch in the counter runs")
    expect_kib = copy_bytes / 1024.0
    f_fetch = expect_kib / fetch[copy[0]]
    f_write = expect_kib / write[copy[0]]
    kernels = {}
    for name in sorted(set(fetch) & set(write)):
        if "rfi::" not in name:
            continue
        kib_r, kib_w = fetch[name], write[name]
        kernels[name] = {
            "fetch_kib": round(kib_r, 1), "write_kib": round(kib_w, 1),
            "hbm_bytes_per_launch": int(round((kib_r * f_fetch + kib_w * f_write) * 1024)),
            "trace": stats.get(name),
        }
    bench = None
    if bench_file and os.path.exists(bench_file):
        with open(bench_file) as f:
            lines = [ln for ln in f if ln.strip().startswith("{")]
        bench = json.loads(lines[-1]) if lines else None
    return {
        "kernel_source_sha256": kernel_source_hash(),
        "calibration": {"copy_kernel": copy[0], "copy_bytes": copy_bytes,
                        "fetch_factor": round(f_fetch, 5), "write_factor": round(f_write, 5)},
        "kernels": kernels,
        "trace_stats": stats,
        "bench_line_of_traced_run": bench,
        "commands": commands,
    }


def trace_by_grid(trace_dir):
    """{(kernel, workgroups): [durations ns]} from a kernel trace."""
    out = {}
    for r in _csv(trace_dir, "_kernel_trace.csv"):
        name = r["Kernel_Name"]
        wgs = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        out.setdefault((name, wgs), []).append(dur)
    return out


def write_trace_markdown(trace_dir, title, commands, out, bench_file=None):
    groups = trace_by_grid(trace_dir)
    lines = ["# rocprofv3 kernel trace: " + title, "", "Commands (run from the repository root on one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Launches grouped by kernel and grid (workgroups of 256 threads).", "",
              "| kernel | workgroups | calls | mean us | min us | max us |", "|---|---|---|---|---|---|"]
    for (name, wgs), d in sorted(groups.items(), key=lambda kv: (kv[0][0], kv[0][1])):
        if "rfi::" not in name:
            continue
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| `{short}` | {wgs} | {len(d)} | {statistics.mean(d) / 1e3:.1f} | "
                     f"{min(d) / 1e3:.1f} | {max(d) / 1e3:.1f} |")
    if bench_file and os.path.exists(bench_file):
        with open(bench_file) as f:
            js = [ln for ln in f if ln.strip().startswith("{")]
        if js:
            lines += ["", "Bench line printed by the traced run:", "", "    " + js[-1].strip()]
    lines += ["", "Kernel sources: sha256 " + kernel_source_hash()]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_markdown(summary, out):
    lines = ["# rocprofv3 summary: int8 plain-scale workload (60 x 2^24, window 4096)", ""]
    lines.append("Commands (run from the repository root on one MI355X):")
    lines.append("")
    for c in summary["commands"]:
        lines.append(f"    {c}")
    lines.append("")
    cal = summary["calibration"]
    lines.append(f"Counter calibration on `{cal['copy_kernel']}` ({cal['copy_bytes']} bytes read "
                 f"and written): FETCH_SIZE x {cal['fetch_factor']}, WRITE_SIZE x "
                 f"{cal['write_factor']}.")
    lines.append("")
    lines.append("| kernel | calls | mean us (trace) | FETCH KiB | WRITE KiB | HBM bytes/launch |")
    lines.append("|---|---|---|---|---|---|")
    for name, k in summary["kernels"].items():
        t = k["trace"] or {}
        lines.append(f"| `{name}` | {t.get('calls', '-')} | "
                     f"{t.get('avg_ns', 0) / 1e3:.1f} | {k['fetch_kib']} | {k['write_kib']} | "
                     f"{k['hbm_bytes_per_launch']} |")
    lines.append("")
    b = summary.get("bench_line_of_traced_run")
    if b:
        lines.append("Bench line printed by the traced run (per-mode means from HIP events, "
                     "same process as the trace):")
        lines.append("")
        lines.append("    " + json.dumps({k: b[k] for k in ("value", "ms_per_step", "modes")
                                         if k in b}))
        lines.append("")
    lines.append("```json")
    lines.append(json.dumps({k: summary[k] for k in ("kernel_source_sha256", "calibration",
                                                    "kernels")}, indent=1))
    lines.append("```")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def load_summary(path):
    """The JSON block of a summary written by write_markdown."""
    text = open(path).read()
    a = text.index("```json") + len("```json")
    b = text.index("```", a)
    return json.loads(text[a:b])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--bench", default=None)
    ap.add_argument("--copy-bytes", type=int)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--trace-only", action="store_true")
    ap.add_argument("--title", default="")
    a = ap.parse_args()
    if a.trace_only:
        write_trace_markdown(a.trace, a.title, a.command, a.out, a.bench)
        print(a.out)
        return
    s = summarize(a.trace, a.fetch, a.write, a.bench, a.copy_bytes, a.command)
    write_markdown(s, a.out)
    print(a.out)


if __name__ == "__main__":
    main()
