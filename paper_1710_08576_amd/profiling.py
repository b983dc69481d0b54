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


def _code_only(text: str) -> str:
    """The source with its comments removed and whitespace collapsed."""
    out = []
    i, n = 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(root: str = HERE) -> str:
    """sha256 of the kernel sources' code: comments and layout do not count,
    so a profile stays valid across an edit of comments alone."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(root, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
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


def counter_passes(dirs):
    """{kernel: {counter: mean value per dispatch}} over counter-pass dirs."""
    per = {}
    for d in dirs:
        for r in _csv(d, "_counter_collection.csv"):
            k = r["Kernel_Name"]
            per.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: statistics.mean(v) for c, v in cs.items()} for k, cs in per.items()}


def derived(c, n_cu=256, n_xcd=8):
    """Ratios of one kernel's counters (None where a counter is missing).
    GRBM_GUI_ACTIVE is summed over the XCDs, so the dispatch's duration in
    cycles is GRBM_GUI_ACTIVE / n_xcd, and its CU-cycles that times n_cu.
      valu_util: SIMD issue time spent on VALU, SQ_ACTIVE_INST_VALU (quad-
        cycles, one per wave64 VALU instruction) x 4 / (4 n_cu x cycles);
      lds_util: CU time the LDS works on indexed operations
        (SQ_LDS_IDX_ACTIVE / CU-cycles);
      lds_bank_conflict, lds_addr_conflict: CU time the LDS stalls on bank
        and address conflicts (SQ_LDS_BANK_CONFLICT, SQ_LDS_ADDR_CONFLICT
        over CU-cycles);
      lds_issue_wait: wave time spent waiting to issue an LDS instruction
        (SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES)."""
    out = {}
    if c.get("GRBM_GUI_ACTIVE"):
        cyc = c["GRBM_GUI_ACTIVE"] / n_xcd
        cu = cyc * n_cu
        out["cycles"] = round(cyc)
        if "SQ_ACTIVE_INST_VALU" in c:
            out["valu_util"] = round(c["SQ_ACTIVE_INST_VALU"] * 4 / (4 * cu), 4)
        for key, name in (("lds_util", "SQ_LDS_IDX_ACTIVE"), ("lds_bank_conflict", "SQ_LDS_BANK_CONFLICT"),
                          ("lds_addr_conflict", "SQ_LDS_ADDR_CONFLICT")):
            if name in c:
                out[key] = round(c[name] / cu, 4)
    if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_LDS" in c:
        out["lds_issue_wait"] = round(c["SQ_WAIT_INST_LDS"] / c["SQ_WAVE_CYCLES"], 4)
    return out


def write_workload_markdown(title, commands, trace_dir, fetch_dir, write_dir, copy_bytes, pmc_dirs,
                            out, run_file=None, units=None):
    """Summary of one workload: trace, calibrated FETCH/WRITE bytes and SQ
    counters per kernel.  units: {kernel substring: (count, what)} to print
    counters per work unit (e.g. per 16 KiB tile)."""
    if not copy_bytes and run_file and os.path.exists(run_file):
        with open(run_file) as f:
            js = [ln for ln in f if ln.strip().startswith("{")]
        copy_bytes = json.loads(js[-1])["copy"]["bytes"]
    s = summarize(trace_dir, fetch_dir, write_dir, None, copy_bytes, commands)
    sq = counter_passes(pmc_dirs) if pmc_dirs else {}
    for name, k in s["kernels"].items():
        if name in sq:
            k["counters"] = {c: round(v, 1) for c, v in sorted(sq[name].items())}
            k["derived"] = derived(sq[name])
            for sub, (n, what) in (units or {}).items():
                if sub in name and n:
                    k["per_" + what] = {c: round(sq[name][c] / n, 2) for c in
                                        ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_WAVES")
                                        if c in sq[name]}
    lines = ["# rocprofv3 summary: " + title, "", "Commands (run from the repository root on one MI355X):", ""]
    lines += ["    " + c for c in commands]
    cal = s["calibration"]
    lines += ["", f"Counter calibration on `{cal['copy_kernel']}` ({cal['copy_bytes']} bytes read and "
                  f"written): FETCH_SIZE x {cal['fetch_factor']}, WRITE_SIZE x {cal['write_factor']}.", "",
              "| kernel | calls | mean us (trace) | HBM bytes/launch | VALU util | LDS util | "
              "LDS bank-conflict | LDS addr-conflict | LDS issue wait |",
              "|---|---|---|---|---|---|---|---|---|"]
    for name, k in s["kernels"].items():
        t = k["trace"] or {}
        dv = k.get("derived", {})
        short = name.replace("(anonymous namespace)::", "").split("(rfi::")[0]
        lines.append(f"| `{short}` | {t.get('calls', '-')} | {t.get('avg_ns', 0) / 1e3:.1f} | "
                     f"{k['hbm_bytes_per_launch']} | {dv.get('valu_util', '-')} | {dv.get('lds_util', '-')} | "
                     f"{dv.get('lds_bank_conflict', '-')} | {dv.get('lds_addr_conflict', '-')} | "
                     f"{dv.get('lds_issue_wait', '-')} |")
    lines += ["", "Dispatch cycles = GRBM_GUI_ACTIVE / 8 (the counter is summed over the 8 XCDs). "
                  "VALU util: SIMD issue time on VALU (SQ_ACTIVE_INST_VALU x 4 over 1024 SIMDs x cycles); "
                  "LDS util, bank- and address-conflict: CU time the LDS works on indexed operations or "
                  "stalls on conflicts (SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT, SQ_LDS_ADDR_CONFLICT over "
                  "256 CUs x cycles); LDS issue wait: wave time waiting to issue an LDS instruction "
                  "(SQ_WAIT_INST_LDS over SQ_WAVE_CYCLES).  Per-tile instruction counts are wave "
                  "instructions summed over the tile's waves."]
    if run_file and os.path.exists(run_file):
        with open(run_file) as f:
            js = [ln for ln in f if ln.strip().startswith("{")]
        if js:
            lines += ["", "Line printed by the traced run (HIP-event medians):", "", "    " + js[-1].strip()]
    lines += ["", "```json", json.dumps({k: s[k] for k in ("kernel_source_sha256", "calibration", "kernels")},
                                        indent=1), "```"]
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
    ap.add_argument("--pmc", action="append", default=[], help="directory of an extra counter pass")
    ap.add_argument("--units", action="append", default=[],
                    help="KERNEL_SUBSTRING=COUNT:WHAT, counters per work unit")
    a = ap.parse_args()
    if a.pmc:
        units = {}
        for u in a.units:
            sub, rest = u.split("=", 1)
            n, what = rest.split(":", 1)
            units[sub] = (int(n), what)
        write_workload_markdown(a.title, a.command, a.trace, a.fetch, a.write, a.copy_bytes, a.pmc, a.out,
                                a.bench, units)
        print(a.out)
        return
    if a.trace_only:
        write_trace_markdown(a.trace, a.title, a.command, a.out, a.bench)
        print(a.out)
        return
    s = summarize(a.trace, a.fetch, a.write, a.bench, a.copy_bytes, a.command)
    write_markdown(s, a.out)
    print(a.out)


if __name__ == "__main__":
    main()
