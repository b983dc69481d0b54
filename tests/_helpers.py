"""Shared helpers for the parity tests: run a batch on the GPU through the
C ABI and on the CPU oracle, on the same seeded bytes, and compare."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

SENTINEL = 0x5A


def unpack(specs):
    return ([s.length for s in specs], [s.window for s in specs], [s.k for s in specs],
            [s.mode for s in specs])


def gpu_run(x_cpu, specs, seed, dev, schedule=None, graph=False, inplace=False, stats=True,
            repeat=1, tpw=None):
    """Run on the device; returns (y numpy, stats structured numpy or None)."""
    L, W, K, M = unpack(specs)
    xd = x_cpu.to(dev)
    fill = SENTINEL if xd.dtype == torch.int8 else 0x5A5A
    yd = xd if inplace else torch.full_like(xd, fill)
    if schedule is None and not graph and tpw is None:
        assert not (inplace and repeat > 1)
        for _ in range(repeat):
            _, st = rfi.mad_filter(xd, L, W, K, M, seed=seed, y=yd, stats=stats)
    else:
        plan = rfi.Plan(x_cpu.element_size(), L, W, K, M, seed=seed)
        if schedule is not None:
            plan.set_schedule(schedule)
        if tpw is not None:
            plan.set_tiles_per_wg(tpw)
        plan.set_graph(graph)
        st = torch.full((max(plan.n_windows, 1), 4), -7, dtype=torch.int32, device=dev) if stats else None
        stream = torch.cuda.Stream() if graph else None
        for _ in range(repeat):
            if stream is not None:
                stream.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(stream):
                    plan.execute(xd, yd, st, stream=stream)
                torch.cuda.current_stream().wait_stream(stream)
            else:
                plan.execute(xd, yd, st)
        torch.cuda.synchronize()
        plan.close()
        st = st[:plan.n_windows] if st is not None else None
    torch.cuda.synchronize()
    return yd.cpu().numpy(), (rfi.stats_numpy(st) if st is not None else None)


def check_against_oracle(x_cpu, specs, seed, y, st, check_padding=True):
    L, W, K, M = unpack(specs)
    xn = x_cpu.numpy()
    yo, sto = oracle.filter_batch(xn, L, W, K, M, seed=seed)
    so, _, _, total = rfi.layout(L, W)
    for s, (o, n) in enumerate(zip(so, L)):
        a, b = y[o:o + n], yo[o:o + n]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(
                f"stream {s} (W={W[s]}, mode={M[s]}, k={K[s]}): {len(bad)} samples differ, "
                f"first at {bad[0]}: gpu {a[bad[0]]} oracle {b[bad[0]]} x {xn[o + bad[0]]}")
        if check_padding:
            pad_end = o + synth.align_up(n)
            assert np.all(y[o + n:pad_end].view(np.uint8 if y.dtype == np.int8 else np.uint16)
                          == (SENTINEL if y.dtype == np.int8 else 0x5A5A)), f"padding of stream {s} written"
    if st is not None:
        if not np.array_equal(st, sto):
            bad = np.nonzero(st != sto)[0]
            raise AssertionError(f"{len(bad)} stats differ, first window {bad[0]}: "
                                 f"gpu {st[bad[0]]} oracle {sto[bad[0]]}")
    return yo, sto
