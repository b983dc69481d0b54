"""Benchmark: Gsamples/s of windowed median/MAD RFI excision on one MI355X.

Workload (the plain-at-scale configuration): 60 int8 streams (30 antennas x
2 polarisations) x 2^24 samples, sigma U[6,20] Gaussian plus impulsive bursts
on 0.1-2 % of samples, window 4096, k = 3.  One step filters the whole batch
once in each replacement mode (zero, clip, noise -- each mode is its own
launch over the full batch), so value = 3 * 60 * 2^24 samples / step time.
Inputs are drawn on the device before timing and stay resident in HBM.

Prints one JSON line.  Extra keys: per-mode rates, the W = 16384 variant,
the roofline of the dominant kernel (HIP events on the launch stream) and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_STREAMS = 60
LENGTH = 1 << 24
HBM_PEAK_GBS = 8000.0
MODE_NAMES = {0: "zero", 1: "clip", 2: "noise"}


def algorithmic_bytes(n_samples: int, n_windows: int, elem: int = 1) -> int:
    """One read and one write per sample, 16 B of statistics per window."""
    return 2 * elem * n_samples + 16 * n_windows


def measured_traffic(kernel_substr: str):
    """Calibrated HBM bytes per launch of a kernel from a committed rocprofv3
    summary under profiles/, if that summary was taken on the current kernel
    sources; else (None, None)."""
    import glob

    from paper_1710_08576_amd import profiling
    cur = profiling.kernel_source_hash()
    for fn in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        try:
            summ = profiling.load_summary(fn)
        except (ValueError, OSError):
            continue
        if summ.get("kernel_source_sha256") != cur:
            continue
        for name, k in summ.get("kernels", {}).items():
            if kernel_substr in name:
                return k["hbm_bytes_per_launch"], os.path.relpath(fn, ROOT)
    return None, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--window", type=int, default=4096)
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the W=16384 variant")
    ap.add_argument("--with-copy", action="store_true",
                    help="after timing, run the HBM copy microbenchmark on the same buffers "
                         "(a kernel of known traffic, to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(streams shard across GPUs with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rfi.load()

    specs = synth.plain_scale(N_STREAMS, LENGTH, args.window, rfi.CLIP)
    x = synth.gen_packed(specs, seed=0, tag=1000, device=dev)
    y = torch.empty_like(x)
    L = [s.length for s in specs]

    def setup(window):
        nw = rfi.layout(L, [window] * N_STREAMS)[2]
        st = torch.empty((nw, 4), dtype=torch.int32, device=dev)
        plans = {}
        for m in (0, 1, 2):
            p = rfi.Plan(1, L, [window] * N_STREAMS, [3.0] * N_STREAMS, [m] * N_STREAMS, seed=1)
            if args.schedule != "auto":
                p.set_schedule(args.schedule)
            plans[m] = p
        return st, plans, nw

    def run_steps(plans, x, y, st, steps, events=None):
        stream = torch.cuda.current_stream()
        for _ in range(steps):
            for m in (0, 1, 2):
                if events is not None:
                    events[m][0].append(torch.cuda.Event(enable_timing=True))
                    events[m][1].append(torch.cuda.Event(enable_timing=True))
                    events[m][0][-1].record(stream)
                plans[m].execute(x, y, st, stream=stream)
                if events is not None:
                    events[m][1][-1].record(stream)

    st, plans, nw = setup(args.window)
    n_samples = N_STREAMS * LENGTH
    run_steps(plans, x, y, st, args.warmup)
    torch.cuda.synchronize()
    events = {m: ([], []) for m in (0, 1, 2)}
    t0 = time.perf_counter()
    run_steps(plans, x, y, st, args.steps, events)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    per_mode_ms = {m: float(np.mean([a.elapsed_time(b) for a, b in zip(*events[m])]))
                   for m in (0, 1, 2)}
    value = 3 * n_samples / (wall / args.steps) / 1e9
    # Dominant kernel: the mode launch with the largest mean duration.
    dom = max(per_mode_ms, key=per_mode_ms.get)
    launches = {m: plans[m].info()["launches"] for m in (0, 1, 2)}
    abytes = algorithmic_bytes(n_samples, nw)
    achieved = abytes / (per_mode_ms[dom] * 1e-3) / 1e9
    # The launch is one tile kernel: class of the window, the mode's bit,
    # one 16 KiB tile per workgroup.
    cls = {512: 0, 1024: 1, 2048: 2, 4096: 3, 8192: 4, 16384: 5}[args.window]
    traffic, traffic_src = measured_traffic("k_i8_tiles<%d, %d, false, 1>" % (cls, 1 << dom))
    modes = {MODE_NAMES[m]: {"ms": round(per_mode_ms[m], 4),
                             "gsamples_s": round(n_samples / per_mode_ms[m] / 1e6, 1),
                             "gb_s": round(abytes / per_mode_ms[m] / 1e6, 1),
                             "launches": launches[m]}
             for m in (0, 1, 2)}
    out = {
        "metric": "Gsamples/s filtered (int8, win 4096, 60 streams)",
        "value": round(value, 2),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic: Gaussian sigma U[6,20] + impulsive bursts, drawn on device",
        "config": {"workload": "plain-scale: 60 streams x 2^24 int8, window %d, k 3, "
                               "zero+clip+noise each over the full batch per step" % args.window,
                   "streams": N_STREAMS, "samples_per_stream": LENGTH, "window": args.window,
                   "k": 3.0, "schedule": plans[0].schedule()},
        "modes": modes,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "calibrated on the copy kernel)",
                     "traffic_source": traffic_src,
                     "kernel": "k_i8_tiles<%d, %d, false, 1> (mode %s)" % (cls, 1 << dom, MODE_NAMES[dom]),
                     "algorithmic_bytes_per_launch": abytes},
    }

    if args.with_copy:
        for _ in range(args.steps):
            rfi._lib.ubench_copy(x, y, 1)
        torch.cuda.synchronize()

    # W = 16384 variant of the same workload (context, not the headline).
    if not args.no_extra:
        st16, plans16, nw16 = setup(16384)
        run_steps(plans16, x, y, st16, 2)
        torch.cuda.synchronize()
        ev16 = {m: ([], []) for m in (0, 1, 2)}
        run_steps(plans16, x, y, st16, max(5, args.steps // 5), ev16)
        torch.cuda.synchronize()
        ms16 = {MODE_NAMES[m]: float(np.mean([a.elapsed_time(b) for a, b in zip(*ev16[m])]))
                for m in (0, 1, 2)}
        out["window_16384"] = {k: {"ms": round(v, 4), "gsamples_s": round(n_samples / v / 1e6, 1)}
                               for k, v in ms16.items()}
        for p in plans16.values():
            p.close()

    # CPU oracle on a bounded sample: whole streams, cycling the modes.
    if not args.no_cpu_baseline:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        so, _, _, _ = rfi.layout([LENGTH] * N_STREAMS, [args.window] * N_STREAMS)
        done, spent, s = 0, 0.0, 0
        while spent < args.cpu_seconds and s < N_STREAMS:
            o = int(so[s])
            xs = x[o:o + LENGTH].cpu().numpy()
            t = time.perf_counter()
            oracle.filter_batch(xs, [LENGTH], [args.window], 3.0, s % 3, seed=1, n_threads=threads)
            spent += time.perf_counter() - t
            done += LENGTH
            s += 1
        out["cpu_baseline"] = {"value": round(done / spent / 1e9, 4), "unit": "Gsamples/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "%d of the %d streams (2^24 int8 each, window %d, k 3), "
                                         "modes zero/clip/noise in turn" % (s, N_STREAMS, args.window)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
