"""Benchmark: Gsamples/s of windowed median/MAD RFI excision on one MI355X.

Workload (the plain-at-scale configuration): 60 int8 streams (30 antennas x
2 polarisations) x 2^24 samples, sigma U[6,20] Gaussian plus impulsive bursts
on 0.1-2 % of samples, window 4096, k = 3.  One step filters the whole batch
once in each replacement mode (zero, clip, noise -- each mode is its own
launch over the full batch), so value = 3 * 60 * 2^24 samples / step time.
Inputs are drawn on the device before timing and stay resident in HBM.

Prints one JSON line.  Extra keys: per-mode rates, the W = 16384 variant,
the roofline of the dominant kernel (HIP events on the launch stream), the
CPU oracle timed on a bounded sample of the same workload, and the other
workloads of the method:

* batching: 64 uneven int8 streams (L U[2^18, 2^24], W from 512..16384,
  k U[2.5, 5], mixed modes) as one plain launch per stream versus one
  batched launch (persistent, fused, graph-replayed; and the autotuned pick);
* int16: 60 x 2^23 int16 samples, window 8192, noise replacement;
* serving: 60 int8 streams, 2^20-sample blocks arriving as Poisson processes
  at the 800 Msample/s real-time rate (mean gap = deadline = 1.31072 ms),
  replayed in real time through the serving runtime; p50/p99 latency from
  arrival to completion against the deadline, plus a run with a block size
  that is no multiple of any window (carry-over) and a saturated run with
  every block ready at once (serving throughput).
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
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-int16", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-mom", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--no-analysis", action="store_true",
                    help="skip the improvement-metric and MAD-breakdown sections")
    ap.add_argument("--no-lds", action="store_true", help="skip the LDS histogram-rate microbenchmark")
    ap.add_argument("--serve-blocks", type=int, default=10000,
                    help="blocks per stream in the real-time serving replay")
    ap.add_argument("--with-copy", action="store_true",
                    help="after timing, run the HBM copy microbenchmark on the same buffers "
                         "(a kernel of known traffic, to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: there is no multi-GPU path (streams would shard "
              "across GPUs with no exchange)", file=sys.stderr)
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
    med_ms = {m: float(np.median([a.elapsed_time(b) for a, b in zip(*events[m])])) for m in (0, 1, 2)}
    modes = {MODE_NAMES[m]: {"ms": round(per_mode_ms[m], 4), "ms_median": round(med_ms[m], 4),
                             "gsamples_s": round(n_samples / per_mode_ms[m] / 1e6, 1),
                             "gb_s": round(abytes / per_mode_ms[m] / 1e6, 1),
                             "launches": launches[m]}
             for m in (0, 1, 2)}
    out = {
        "metric": "Gsamples/s filtered (int8, win 4096, 60 streams) + %HBM roofline; p99 block latency",
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

    # Streaming ceiling of this GPU: the copy microbenchmark on the same
    # buffers (one read and one write per byte, the kernels' access shape).
    stream = torch.cuda.current_stream()
    copy_ms = _time_events(lambda: rfi._lib.ubench_copy(x, y, 1), max(10, args.steps // 2), stream)
    copy_gbs = 2 * x.numel() / copy_ms / 1e6
    out["roofline"]["copy_ceiling"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if args.with_copy:
        for _ in range(args.steps):
            rfi._lib.ubench_copy(x, y, 1)
        torch.cuda.synchronize()

    # Other windows of the same workload (context, not the headline): each
    # plan warmed like the headline's, then timed per launch; median and mean
    # both reported (a rare stall on the box moves the mean only).
    def side_window(window):
        stw, plansw, nww = setup(window)
        run_steps(plansw, x, y, stw, args.warmup)
        torch.cuda.synchronize()
        evw = {m: ([], []) for m in (0, 1, 2)}
        run_steps(plansw, x, y, stw, max(10, args.steps // 2), evw)
        torch.cuda.synchronize()
        abw = algorithmic_bytes(n_samples, nww)
        res = {}
        for m in (0, 1, 2):
            t = [a.elapsed_time(b) for a, b in zip(*evw[m])]
            v = float(np.median(t))
            res[MODE_NAMES[m]] = {
                "ms_median": round(v, 4), "ms": round(float(np.mean(t)), 4),
                "gsamples_s": round(n_samples / v / 1e6, 1), "gb_s": round(abw / v / 1e6, 1),
                "roofline_frac": round(abw / v / 1e6 / HBM_PEAK_GBS, 4),
                "launches": plansw[m].info()["launches"]}
        res["schedule"] = plansw[0].schedule()
        for p in plansw.values():
            p.close()
        del stw
        return res

    if not args.no_extra:
        out["window_16384"] = side_window(16384)
        # W = 5000, not a tile class: every window through the generic
        # kernel (register-resident, one window per workgroup).
        out["window_5000_generic"] = side_window(5000)

    if not args.no_batching:
        out["batching"] = bench_batching(args, dev)
    if not args.no_int16:
        out["int16"] = bench_int16(args, dev)
    if not args.no_mom:
        out["median_of_mad"] = bench_mom(args, dev, x, y, L)
    if not args.no_multi:
        out["three_outputs_per_call"] = bench_multi(args, dev, x, L)
    if not args.no_analysis:
        out["improvement_metric"] = bench_improvement(args, dev, x, y, L)
        out["mad_breakdown"] = bench_breakdown(args, dev)
    if not args.no_lds:
        out["lds_atomic_rate"] = bench_lds(args, dev, x)
    if not args.no_serving:
        del x, y
        torch.cuda.empty_cache()
        out["serving"] = bench_serving(args, dev)
        out["p99_block_latency_ms"] = out["serving"]["realtime"]["p99_ms"]
        x = synth.gen_packed(specs, seed=0, tag=1000, device=dev)

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
                               "cores": threads, "kind": "oracle", "cpu_model": _cpu_model(),
                               "host_cpus": os.cpu_count(),
                               "sample": "%d of the %d streams (2^24 int8 each, window %d, k 3), "
                                         "modes zero/clip/noise in turn" % (s, N_STREAMS, args.window)}
    print(json.dumps(out))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _time_events(fn, iters, stream):
    """Median ms of fn() over iters runs, HIP events on `stream` (the
    median: a rare stall of tens of milliseconds on the box would otherwise
    dominate a mean over ten runs)."""
    import numpy as np
    import torch
    evs = []
    for _ in range(iters):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def bench_batching(args, dev):
    """One launch per stream versus the batched launch, same buffers."""
    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import synth
    specs = synth.batching()
    L = [s.length for s in specs]
    W = [s.window for s in specs]
    K = [s.k for s in specs]
    M = [s.mode for s in specs]
    x = synth.gen_packed(specs, seed=0, tag=2000, device=dev)
    y = torch.empty_like(x)
    nw = rfi.layout(L, W)[2]
    st = torch.empty((nw, 4), dtype=torch.int32, device=dev)
    n = sum(L)
    abytes = algorithmic_bytes(n, nw)
    stream = torch.cuda.Stream()
    iters = max(10, args.steps // 2)
    res = {"workload": "64 int8 streams, L U[2^18,2^24] (%d samples), W 512..16384, "
                       "k U[2.5,5], mixed modes" % n}
    variants = [("per_stream_launches", "per_stream", False), ("batched_fused_persist_graph",
                                                               "fused_persist", True),
                ("batched_split_graph", "split", True),
                ("batched_split_concurrent_graph", "split_concurrent", True),
                ("batched_fused_concurrent_graph", "fused_concurrent", True),
                ("batched_one_launch_graph", "one_launch", True),
                ("batched_one_launch_persist_graph", "one_launch_persist", True)]
    with torch.cuda.stream(stream):
        for name, sched, graph in variants:
            p = rfi.Plan(1, L, W, K, M, seed=3)
            p.set_schedule(sched)
            p.set_graph(graph)
            for _ in range(3):
                p.execute(x, y, st, stream=stream)
            ms = _time_events(lambda: p.execute(x, y, st, stream=stream), iters, stream)
            res[name] = {"ms": round(ms, 4), "gsamples_s": round(n / ms / 1e6, 1),
                         "gb_s": round(abytes / ms / 1e6, 1), "launches": p.info()["launches"]}
            p.close()
        p = rfi.Plan(1, L, W, K, M, seed=3)
        best, best_ms = p.autotune(x, y, st, iters=5, stream=stream)
        p.set_graph(True)
        for _ in range(3):
            p.execute(x, y, st, stream=stream)
        ms = _time_events(lambda: p.execute(x, y, st, stream=stream), iters, stream)
        inv = {v: k for k, v in rfi.SCHEDULES.items()}
        res["batched_autotuned_graph"] = {"ms": round(ms, 4), "gsamples_s": round(n / ms / 1e6, 1),
                                          "gb_s": round(abytes / ms / 1e6, 1),
                                          "schedule": inv.get(best, best),
                                          "launches": p.info()["launches"]}
        p.close()
    base = res["per_stream_launches"]["ms"]
    res["speedup_batched_vs_per_stream"] = round(base / res["batched_autotuned_graph"]["ms"], 3)
    res["roofline_frac_batched"] = round(res["batched_autotuned_graph"]["gb_s"] / HBM_PEAK_GBS, 4)
    return res


def bench_int16(args, dev):
    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import synth
    specs = synth.int16_path()
    L = [s.length for s in specs]
    x = synth.gen_packed(specs, seed=0, tag=3000, device=dev)
    y = torch.empty_like(x)
    nw = rfi.layout(L, [8192] * len(L))[2]
    st = torch.empty((nw, 4), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    n = sum(L)
    ab = algorithmic_bytes(n, nw, elem=2)
    res = {"workload": "60 x 2^23 int16, window 8192, k 3, noise"}
    # noise is the workload; zero and clip of the same batch for context
    for m in (2, 0, 1):
        p = rfi.Plan(2, L, [8192] * len(L), [3.0] * len(L), [m] * len(L), seed=5)
        for _ in range(max(3, args.warmup)):
            p.execute(x, y, st, stream=stream)
        ms = _time_events(lambda: p.execute(x, y, st, stream=stream), max(10, args.steps // 2), stream)
        r = {"ms": round(ms, 4), "gsamples_s": round(n / ms / 1e6, 1), "gb_s": round(ab / ms / 1e6, 1),
             "roofline_frac": round(ab / ms / 1e6 / HBM_PEAK_GBS, 4)}
        p.close()
        if m == 2:
            res.update(r)
        else:
            res.setdefault("other_modes", {})[MODE_NAMES[m]] = r
    return res


def bench_multi(args, dev, x, L):
    """Several outputs of the plain-scale batch from one call (the paper's
    side-by-side comparison of thresholds and replacement options): three
    outputs without noise (zero at k 3 and 5, clip at k 3) share one read of
    the input; zero, clip and noise at k 3 put noise in a pass of its own.
    Each is timed beside the same outputs as single calls."""
    import torch

    import paper_1710_08576_amd as rfi
    ns, n = len(L), sum(L)
    ys = [torch.empty_like(x) for _ in range(3)]
    W = [4096] * ns
    nw = rfi.layout(L, W)[2]
    stream = torch.cuda.current_stream()
    reps = max(10, args.steps // 5)
    out = {}
    for name, kk, mm in (("zero_k3_zero_k5_clip_k3", (3.0, 5.0, 3.0), (0, 0, 1)),
                         ("zero_clip_noise_k3", (3.0, 3.0, 3.0), (0, 1, 2))):
        ks = [[k] * ns for k in kk]
        ms_ = [[m] * ns for m in mm]
        fn = lambda: rfi.mad_filter_multi(x, L, W, ks, ms_, seed=1, ys=ys, stats=False)

        def singles():
            for o in range(3):
                rfi.mad_filter(x, L, W, ks[o], ms_[o], seed=1, y=ys[o], stats=False)
        for _ in range(3):
            fn()
            singles()
        ms = _time_events(fn, reps, stream)
        ms1 = _time_events(singles, reps, stream)
        reads = 1 if 2 not in mm else 2
        ab = (reads + 3) * n
        out[name] = {"ms": round(ms, 4), "reads_of_x": reads, "gb_s": round(ab / ms / 1e6, 1),
                     "roofline_frac": round(ab / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "three_single_calls_ms": round(ms1, 4), "speedup_vs_single_calls": round(ms1 / ms, 3)}
    return {"workload": "plain-scale 60 x 2^24 int8, W 4096, three outputs per call",
            "algorithmic_bytes": "per read of x 1 B/sample, per output 1 B/sample written (no statistics)",
            "windows": nw, **out}


def bench_improvement(args, dev, x, y, L):
    """Improvement metric (Sec. III-A) of each replacement mode on the
    plain-scale batch (W 4096, k 3): power integrated over blocks of 2^20
    samples (1.31 ms at 800 Msample/s, the beamformer's 1.3 ms), S = RMS
    deviation over mean averaged over segments of 16 blocks, and the printed
    improvement 10 log10(S_U / S_F) per stream."""
    import numpy as np
    import torch

    import paper_1710_08576_amd as rfi
    ns, n = len(L), sum(L)
    block, seg = 1 << 20, 16
    W = [4096] * ns
    stream = torch.cuda.current_stream()
    nb = rfi.n_blocks(L, block)
    pu = torch.empty(nb, dtype=torch.int64, device=dev)
    pf = torch.empty(nb, dtype=torch.int64, device=dev)
    res = torch.empty((ns, 3), dtype=torch.float64, device=dev)
    rfi.block_power(x, L, block, out=pu)
    reps = max(10, args.steps // 5)
    ms_pow = _time_events(lambda: rfi.block_power(x, L, block, out=pu), reps, stream)
    ms_imp = _time_events(lambda: rfi.improvement(pu, pf, L, block, seg, out=res), reps, stream)
    ab = n + 8 * nb
    out = {"workload": "plain-scale 60 x 2^24 int8, W 4096, k 3; blocks of 2^20 samples, segments of 16 blocks",
           "block_power": {"ms": round(ms_pow, 4), "gb_s": round(ab / ms_pow / 1e6, 1),
                           "roofline_frac": round(ab / ms_pow / 1e6 / HBM_PEAK_GBS, 4),
                           "algorithmic_bytes": "1 B/sample read + 8 B/block written"},
           "improvement_kernel_ms": round(ms_imp, 4)}
    for name, m in (("zero", 0), ("clip", 1), ("noise", 2)):
        rfi.mad_filter(x, L, W, [3.0] * ns, [m] * ns, seed=1, y=y, stats=False)
        rfi.block_power(y, L, block, out=pf)
        r = rfi.improvement(pu, pf, L, block, seg, out=res).cpu().numpy()
        out[name + "_db"] = {"median": round(float(np.median(r[:, 2])), 2), "min": round(float(r[:, 2].min()), 2),
                             "max": round(float(r[:, 2].max()), 2)}
    out["s_unfiltered_median"] = round(float(np.median(r[:, 0])), 5)
    return out


def bench_breakdown(args, dev):
    """MAD breakdown on emulator bursts (Sec. III-B): 60 streams of 2^24
    int8 samples (sigma U[6, 20]), Gaussian bursts 15 dB above the noise,
    one every 2^22 samples from sample 2^20 on; per burst length the
    fraction of burst samples flagged by MAD with W 16384 and 4096 and by the
    median of MAD (W 4096, 4096 windows), all clip mode (clip changes
    exactly the flagged samples), and the time of each filter."""
    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import synth
    specs = synth.plain_scale(60, 1 << 24, 4096, rfi.CLIP)
    ns, L = len(specs), 1 << 24
    lengths = [L] * ns
    period, phase = 1 << 22, 1 << 20
    so = rfi.layout(lengths, [4096] * ns)[0]
    stream = torch.cuda.current_stream()
    out = {"workload": "emulator bursts: 60 x 2^24 int8, 15 dB Gaussian bursts every 2^22 samples from 2^20; "
                       "on-lengths in samples at 800 Msample/s (51200 = 64 us)"}
    for on in (2048, 8192, 16384, 51200):
        x = torch.zeros(int(so[-1]) + synth.align_up(L), dtype=torch.int8, device=dev)
        for s, sp in enumerate(specs):
            x[so[s]:so[s] + L] = synth.gen_emulator_stream(L, sp.sigma, on, period, phase, 15.0, 0, s, device=dev)
        mask = synth.emulator_mask(L, on, period, phase, device=dev)
        yb = torch.empty_like(x)
        row = {}
        for name, fn in (("mad_w16384", lambda: rfi.mad_filter(x, lengths, [16384] * ns, [3.0] * ns, [1] * ns,
                                                                seed=1, y=yb, stats=False)[0]),
                         ("mad_w4096", lambda: rfi.mad_filter(x, lengths, [4096] * ns, [3.0] * ns, [1] * ns,
                                                              seed=1, y=yb, stats=False)[0]),
                         ("mom_w4096_k4096", lambda: rfi.mom_filter(x, lengths, [4096] * ns, [3.0] * ns, [1] * ns,
                                                                    4096, seed=1, y=yb, stats=False)[0])):
            y = fn()
            flagged = 0
            for s in range(ns):
                flagged += int(((y[so[s]:so[s] + L] != x[so[s]:so[s] + L]) & mask).sum())
            det = flagged / (ns * int(mask.sum()))
            ms = _time_events(fn, 5, stream)
            row[name] = {"detected": round(det, 4), "ms": round(ms, 4)}
        out[f"on_{on}"] = row
        del x, yb
    return out


CU_COUNT, CLOCK_GHZ = 256, 2.4


def bench_lds(args, dev, x):
    """The int8 selection's second roof: LDS atomics per CU per clock of the
    histogram microbenchmark (one atomic per sample, per-wave histograms of
    R replicas), on the plain-scale bytes for R = 1, 2, 4, 8 and on Gaussian
    int8 of several sigma at R = 4 (the tile kernels' choice).  At 70 % of
    8 TB/s the int8 filter needs 2.8 Gsamples/s = 4.6 atomics per CU per
    clock."""
    import torch

    from paper_1710_08576_amd import _lib
    stream = torch.cuda.current_stream()
    hist = torch.zeros((256, 256), dtype=torch.int32, device=dev)
    n = x.numel() // 16384 * 16384
    xs = x[:n]

    def rate(buf, r):
        for _ in range(2):
            _lib.ubench_lds_hist(buf, r, hist=hist)
        ms = _time_events(lambda: _lib.ubench_lds_hist(buf, r, hist=hist), 10, stream)
        return {"ms": round(ms, 4), "atomics_per_cu_clock": round(buf.numel() / (ms * 1e-3) / (CU_COUNT * CLOCK_GHZ * 1e9), 2)}

    out = {"unit": "lane-atomics per CU per clock (256 CUs, 2.4 GHz)", "needed_at_70pct": 4.56,
           "plain_scale": {f"R{r}": rate(xs, r) for r in (1, 2, 4, 8)}}
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    m = 1 << 28
    sweep = {}
    for sigma in (2, 6, 20, 60):
        buf = torch.clamp(torch.round(torch.randn(m, generator=g, device=dev) * sigma), -128, 127).to(torch.int8)
        sweep[f"sigma_{sigma}"] = rate(buf, 4)
        del buf
    buf = torch.randint(-128, 128, (m,), generator=g, dtype=torch.int8, device=dev)
    sweep["uniform"] = rate(buf, 4)
    del buf
    out["gaussian_R4"] = sweep
    return out


def bench_mom(args, dev, x, y, L):
    """Median of MAD (K = 4096 windows of 4096, the paper's setting) on the
    plain-scale batch: statistics pass, median of MADs, replacement pass."""
    import numpy as np
    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import _lib
    n, ns = sum(L), len(L)
    nw = rfi.layout(L, [4096] * ns)[2]
    st = torch.empty((nw, 4), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    Ws = np.full(ns, 4096, dtype=np.int32)
    Ks = np.full(ns, 3.0, dtype=np.float32)
    res = {"workload": "plain-scale 60 x 2^24 int8, W 4096, median of the MADs of 4096 windows, k 3",
           "algorithmic_bytes": "3 B/sample (x read twice, y written once) + 16 B/window"}
    ab = 3 * n + 16 * nw
    for name, m in (("zero", 0), ("clip", 1), ("noise", 2)):
        Ms = np.full(ns, m, dtype=np.int32)

        def fn():
            _lib._check(_lib.load().rfi_mom_filter(
                _lib._tptr(x), _lib._tptr(y), ns, _lib._ptr(Ls), _lib._ptr(Ws), _lib._ptr(Ks),
                _lib._ptr(Ms), 4096, 1, _lib._tptr(st), _lib._stream_handle(stream)), "rfi_mom_filter")
        for _ in range(3):
            fn()
        ms = _time_events(fn, max(10, args.steps // 5), stream)
        res[name] = {"ms": round(ms, 4), "gsamples_s": round(n / ms / 1e6, 1),
                     "gb_s": round(ab / ms / 1e6, 1), "roofline_frac": round(ab / ms / 1e6 / HBM_PEAK_GBS, 4)}
    # Real-time use: one 2^20-sample block of every stream per call, the MAD
    # history (4095 windows) and the sample base carried on the device.
    blk = 1 << 20
    xb = x[:ns * blk].view(ns, blk).contiguous().view(-1)
    yb = torch.empty_like(xb)
    hist = torch.zeros((ns, 4095), dtype=torch.uint8, device=dev)
    hlen = torch.zeros(ns, dtype=torch.int32, device=dev)
    absb = torch.zeros(ns, dtype=torch.int64, device=dev)
    stb = torch.empty((ns * blk // 4096, 4), dtype=torch.int32, device=dev)
    Lb = np.full(ns, blk, dtype=np.int64)
    Mb = np.full(ns, 2, dtype=np.int32)

    def call():
        _lib._check(_lib.load().rfi_mom_filter_carry(
            _lib._tptr(xb), _lib._tptr(yb), ns, _lib._ptr(Lb), _lib._ptr(Ws), _lib._ptr(Ks), _lib._ptr(Mb), 4096, 1,
            _lib._tptr(absb), _lib._tptr(hist), _lib._tptr(hlen), _lib._tptr(stb), _lib._stream_handle(stream)),
            "rfi_mom_filter_carry")
        absb.add_(blk)
    for _ in range(3):
        call()
    ms = _time_events(call, max(10, args.steps // 5), stream)
    res["carried_blocks_noise"] = {"workload": "60 streams, one 2^20-sample block each per call, history of 4095 MADs "
                                               "carried on the device, noise",
                                   "ms_per_call": round(ms, 4), "deadline_ms": round(DEADLINE_NS / 1e6, 5),
                                   "gsamples_s": round(ns * blk / ms / 1e6, 1)}
    return res


DEADLINE_NS = (1 << 20) / 800e6 * 1e9  # one 2^20-sample block at 800 Msample/s


def bench_serving(args, dev):
    """Real-time replay through the serving runtime (see module docstring)."""
    import numpy as np
    import torch

    import paper_1710_08576_amd as rfi
    from paper_1710_08576_amd import synth
    specs = synth.serving_streams()
    ns = len(specs)
    ring = 64
    block = 1 << 20
    # ring of pre-generated blocks per stream, resident on the device
    xs = []
    for i, s in enumerate(specs):
        s.length = ring * block
        xs.append(synth.gen_stream(s, 0, 4000, i, device=dev))
    maxw = max(s.window for s in specs)
    outs = torch.empty((ns, ring, block + maxw), dtype=torch.int8, device=dev)
    stats = torch.empty((ns, ring, (block + 2 * maxw) // 512, 4), dtype=torch.int32, device=dev)
    res = {"workload": "60 int8 streams, 2^20-sample blocks, Poisson arrivals at 800 Msample/s "
                       "per stream (mean gap %.5f ms), W %s, k 3, clip" %
                       (DEADLINE_NS / 1e6, sorted({s.window for s in specs})),
           "deadline_ms": DEADLINE_NS / 1e6}

    def run(n_per_stream, blen, arrivals):
        srv = rfi.Server(elem_size=1, max_streams=ns, max_inflight=1024, max_batch=64,
                         hbm_budget_bytes=2 << 30, seed=7, n_lanes=4, schedule="fused")
        for i, s in enumerate(specs):
            srv.add_stream(i, s.window, s.k, s.mode)
        sid = np.repeat(np.arange(ns, dtype=np.uint32)[None, :], n_per_stream, 0)
        blk = np.repeat(np.arange(n_per_stream)[:, None], ns, 1)
        t = arrivals(n_per_stream)
        order = np.argsort(t.ravel(), kind="stable")
        sid, blk, t = sid.ravel()[order], blk.ravel()[order], t.ravel()[order]
        slot = blk % ring
        # blocks of length blen tile the ring's stream buffer (wrapping)
        start = (blk % ((ring * block) // blen)) * blen
        bptr = np.array([xs[i].data_ptr() for i in range(ns)], np.uint64)[sid] + start.astype(np.uint64)
        optr = (np.uint64(outs.data_ptr()) + ((sid.astype(np.uint64) * ring + slot.astype(np.uint64))
                                              * np.uint64(outs.shape[2])))
        sptr = (np.uint64(stats.data_ptr()) + ((sid.astype(np.uint64) * ring + slot.astype(np.uint64))
                                               * np.uint64(stats.shape[2] * 16)))
        # 16-byte alignment of the block addresses
        assert np.all(bptr % 16 == 0) and np.all(optr % 16 == 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, em = srv.replay_ptrs(sid, t, bptr, optr, np.full(len(sid), blen), sptr)
        wall = time.perf_counter() - t0
        c = srv.counters()
        srv.close()
        lat_ms = lat / 1e6
        n_blocks = len(sid)
        r = {"blocks": int(n_blocks), "block_samples": blen,
             "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
             "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
             "p999_ms": round(float(np.percentile(lat_ms, 99.9)), 4),
             "max_ms": round(float(lat_ms.max()), 4),
             "deadline_misses": int((lat > DEADLINE_NS).sum()),
             "gsamples_s": round(n_blocks * blen / wall / 1e9, 2),
             "launches": c["launches"], "refused": c["refused"],
             "ticket_records_live_peak": c["live_peak"], "ticket_records_live_at_end": c["live_records"]}
        return r

    def poisson(n):
        rng = np.random.default_rng(11)
        gaps = rng.exponential(DEADLINE_NS, size=(n, ns))
        return np.cumsum(gaps, 0).astype(np.int64)

    res["realtime"] = run(args.serve_blocks, block, poisson)
    res["realtime_carry"] = run(max(200, args.serve_blocks // 5), 1_000_000, poisson)
    res["saturated"] = run(200, block, lambda n: np.zeros((n, ns), np.int64))
    return res


if __name__ == "__main__":
    main()
