"""Every byte at the sizes the benchmark measures: each workload is filtered
on the device in the launch configuration the benchmark times and compared
element by element, output samples and per-window statistics, with the
oracle run on the host over the same bytes (Sec. II-D, Eqs. (1)-(3)).

- plain-scale, 60 x 2^24 int8, W 4096 and 16384, each mode;
- int16, 60 x 2^23, W 8192, noise;
- batching, 64 uneven streams (W 512..16384, mixed k and modes), the
  autotuned schedule replayed from a HIP graph;
- median of MAD on the plain-scale batch, W 4096, K 4096, each mode.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

pytestmark = pytest.mark.gpu


def _compare(y_dev, st_dev, yo, sto, lengths, windows, what):
    so, _, nw, _ = rfi.layout(lengths, windows)
    y = y_dev.cpu().numpy()
    for s, (o, n) in enumerate(zip(so, lengths)):
        a, b = y[o:o + n], yo[o:o + n]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{what}: stream {s}: {len(bad)} samples differ, first at {bad[0]} "
                                 f"(gpu {a[bad[0]]}, oracle {b[bad[0]]})")
    st = rfi.stats_numpy(st_dev[:nw])
    if not np.array_equal(st, sto):
        bad = np.nonzero(st != sto)[0]
        raise AssertionError(f"{what}: {len(bad)} of {nw} statistics differ, first window {bad[0]}: "
                             f"gpu {st[bad[0]]} oracle {sto[bad[0]]}")


@pytest.mark.parametrize("W", [4096, 16384])
@pytest.mark.parametrize("mode", [rfi.ZERO, rfi.CLIP, rfi.NOISE])
def test_plain_scale_every_byte(gpu, W, mode):
    # the benchmark's batch (seed 0, tag 1000) and plans (Philox seed 1)
    specs = synth.plain_scale(60, 1 << 24, W, rfi.CLIP)
    L = [s.length for s in specs]
    x = synth.gen_packed(specs, seed=0, tag=1000, device=gpu)
    nw = rfi.layout(L, [W] * 60)[2]
    y = torch.empty_like(x)
    st = torch.full((nw, 4), -1, dtype=torch.int32, device=gpu)
    p = rfi.Plan(1, L, [W] * 60, [3.0] * 60, [mode] * 60, seed=1)
    p.execute(x, y, st)
    torch.cuda.synchronize()
    p.close()
    xh = x.cpu().numpy()
    del x
    yo, sto = oracle.filter_batch(xh, L, [W] * 60, 3.0, mode, seed=1)
    _compare(y, st, yo, sto, L, [W] * 60, f"plain-scale W {W} mode {mode}")


def test_int16_every_byte(gpu):
    specs = synth.int16_path()
    L = [s.length for s in specs]
    W = [8192] * len(L)
    x = synth.gen_packed(specs, seed=0, tag=3000, device=gpu)
    nw = rfi.layout(L, W)[2]
    y = torch.empty_like(x)
    st = torch.full((nw, 4), -1, dtype=torch.int32, device=gpu)
    p = rfi.Plan(2, L, W, [3.0] * len(L), [rfi.NOISE] * len(L), seed=5)
    p.execute(x, y, st)
    torch.cuda.synchronize()
    p.close()
    xh = x.cpu().numpy()
    del x
    yo, sto = oracle.filter_batch(xh, L, W, 3.0, rfi.NOISE, seed=5)
    _compare(y, st, yo, sto, L, W, "int16 W 8192 noise")


def test_batching_every_byte_autotuned_graph(gpu):
    specs = synth.batching()
    L, W = [s.length for s in specs], [s.window for s in specs]
    K, M = [s.k for s in specs], [s.mode for s in specs]
    x = synth.gen_packed(specs, seed=0, tag=2000, device=gpu)
    nw = rfi.layout(L, W)[2]
    y = torch.empty_like(x)
    st = torch.empty((nw, 4), dtype=torch.int32, device=gpu)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    p = rfi.Plan(1, L, W, K, M, seed=3)
    with torch.cuda.stream(stream):
        p.autotune(x, y, st, iters=3, stream=stream)
        p.set_graph(True)
        for _ in range(2):  # capture, then a replay
            y.fill_(0x5A)
            st.fill_(-1)
            p.execute(x, y, st, stream=stream)
    torch.cuda.synchronize()
    p.close()
    xh = x.cpu().numpy()
    del x
    yo, sto = oracle.filter_batch(xh, L, W, K, M, seed=3)
    _compare(y, st, yo, sto, L, W, "batching, autotuned schedule, graph replay")


@pytest.mark.parametrize("mode", [rfi.ZERO, rfi.CLIP, rfi.NOISE])
def test_median_of_mad_every_byte(gpu, mode):
    specs = synth.plain_scale(60, 1 << 24, 4096, rfi.CLIP)
    L = [s.length for s in specs]
    W = [4096] * 60
    x = synth.gen_packed(specs, seed=0, tag=1000, device=gpu)
    y, st = rfi.mom_filter(x, L, W, [3.0] * 60, [mode] * 60, 4096, seed=1)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    del x
    yo, sto = oracle.mom_filter_batch(xh, L, W, 3.0, mode, 4096, seed=1)
    _compare(y, st, yo, sto, L, W, f"median of MAD W 4096 K 4096 mode {mode}")
