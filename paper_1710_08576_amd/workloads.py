"""One benchmark workload per process, for profiler passes.

rocprofv3 wraps a whole process, and a counter pass averages every dispatch
of a kernel it sees; running one workload per process keeps each summary to
the launches of that workload alone.  The inputs are the benchmark's
(synthetic, drawn on the device with the same seeds), the launches those the
benchmark times, repeated --reps times after one warm-up.  --with-copy adds
the HBM copy microbenchmark on buffers of the same size, whose known traffic
calibrates the FETCH_SIZE / WRITE_SIZE counters.

Usage:  python -m paper_1710_08576_amd.workloads --workload plain --window 4096
            --modes zero,clip,noise --reps 5 --with-copy
        python -m paper_1710_08576_amd.workloads --workload int16 --reps 5
        python -m paper_1710_08576_amd.workloads --workload batching --schedule fused --reps 5
        python -m paper_1710_08576_amd.workloads --workload batching --autotune-save tune.json
        python -m paper_1710_08576_amd.workloads --workload batching --tune-file tune.json --reps 5

--autotune-save tunes the workload's plan (every schedule timed on its
buffers), writes the autotune table and exits; --tune-file loads such a
table first, so that a later process (a profiled one) runs the tuned
launches alone.
"""
from __future__ import annotations

import argparse
import json

MODES = {"zero": 0, "clip": 1, "noise": 2}


def _time(fn, reps, stream):
    import torch
    evs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    return sorted(a.elapsed_time(b) for a, b in evs)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=["plain", "int16", "batching"])
    ap.add_argument("--window", type=int, default=4096)
    ap.add_argument("--modes", default="zero,clip,noise")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--with-copy", action="store_true")
    ap.add_argument("--autotune-save", default=None)
    ap.add_argument("--tune-file", default=None)
    a = ap.parse_args(argv)

    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import synth
    dev = torch.device("cuda:0")
    rfi.load()
    if a.tune_file:
        rfi.tune_load(a.tune_file)
    stream = torch.cuda.current_stream()
    out = {"workload": a.workload}
    if a.workload == "plain":
        specs = synth.plain_scale(60, 1 << 24, a.window, rfi.CLIP)
        x = synth.gen_packed(specs, seed=0, tag=1000, device=dev)
        L = [s.length for s in specs]
        W = [a.window] * len(L)
        elem, seed, tag = 1, 1, "plain-scale 60 x 2^24 int8, W %d" % a.window
        runs = [(m, [3.0] * len(L), [MODES[m]] * len(L)) for m in a.modes.split(",")]
    elif a.workload == "int16":
        specs = synth.int16_path()
        x = synth.gen_packed(specs, seed=0, tag=3000, device=dev)
        L = [s.length for s in specs]
        W = [8192] * len(L)
        elem, seed, tag = 2, 5, "int16 60 x 2^23, W 8192"
        runs = [(m, [3.0] * len(L), [MODES[m]] * len(L)) for m in a.modes.split(",")]
    else:
        specs = synth.batching()
        x = synth.gen_packed(specs, seed=0, tag=2000, device=dev)
        L = [s.length for s in specs]
        W = [s.window for s in specs]
        elem, seed, tag = 1, 3, "batching, 64 uneven int8 streams"
        runs = [("mixed", [s.k for s in specs], [s.mode for s in specs])]
    y = torch.empty_like(x)
    nw = rfi.layout(L, W)[2]
    st = torch.empty((nw, 4), dtype=torch.int32, device=dev)
    out["config"] = tag
    if a.autotune_save:
        inv = {v: k for k, v in rfi.SCHEDULES.items()}
        for name, K, M in runs:
            p = rfi.Plan(elem, L, W, K, M, seed=seed)
            best, ms = p.autotune(x, y, st, iters=5, stream=stream)
            out[name] = {"autotuned": inv.get(best, best), "ms": round(ms, 4)}
            p.close()
        rfi.tune_save(a.autotune_save)
        print(json.dumps(out), flush=True)
        return
    for name, K, M in runs:
        p = rfi.Plan(elem, L, W, K, M, seed=seed)
        if a.schedule != "auto":
            p.set_schedule(a.schedule)
        p.set_graph(a.workload == "batching")
        p.execute(x, y, st, stream=stream)
        ts = _time(lambda: p.execute(x, y, st, stream=stream), a.reps, stream)
        out[name] = {"ms_median": round(ts[len(ts) // 2], 4), "schedule": p.schedule(),
                     "launches": p.info()["launches"]}
        p.close()
    if a.with_copy:
        # the copy kernel takes whole 16 KiB tiles: the largest such prefix
        nb = (x.numel() * x.element_size()) // 16384 * 16384
        xb, yb = x.view(torch.uint8)[:nb], y.view(torch.uint8)[:nb]
        rfi._lib.ubench_copy(xb, yb, 1)
        ts = _time(lambda: rfi._lib.ubench_copy(xb, yb, 1), a.reps, stream)
        out["copy"] = {"bytes": nb, "ms_median": round(ts[len(ts) // 2], 4)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
