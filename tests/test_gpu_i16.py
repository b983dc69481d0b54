"""int16 parity: radix-select path through the C ABI against the CPU oracle,
bit-exact in output samples and per-window statistics."""
import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

from _helpers import check_against_oracle, gpu_run, unpack

pytestmark = pytest.mark.gpu

MODES = [rfi.ZERO, rfi.CLIP, rfi.NOISE]


@pytest.mark.parametrize("mode", MODES)
def test_w8192_tiles_and_tail(gpu, mode):
    specs = [synth.StreamSpec(8192 * 5 + 3001 + 19 * s, 8192, 3.0, mode, 400.0, 0.01, 32, 32, "i16")
             for s in range(3)]
    x = synth.gen_packed(specs, seed=1, tag=20)
    y, st = gpu_run(x, specs, 8, gpu)
    check_against_oracle(x, specs, 8, y, st)


@pytest.mark.parametrize("W", [1, 2, 5, 100, 1024, 4096, 5000, 16384, 65536])
@pytest.mark.parametrize("mode", MODES)
def test_generic_windows(gpu, W, mode):
    L = max(2 * W + W // 2 + 3, 200)
    specs = [synth.StreamSpec(L, W, 2.5, mode, 400.0, 0.02, 16, 64, "i16"),
             synth.StreamSpec(L // 3 + 1, W, 4.0, mode, 30.0, 0.01, 16, 64, "i16")]
    x = synth.gen_packed(specs, seed=W, tag=21)
    y, st = gpu_run(x, specs, 6, gpu)
    check_against_oracle(x, specs, 6, y, st)


@pytest.mark.parametrize("k", [0.0, 0.5, 1.0])
def test_w8192_noise_many_flagged(gpu, k):
    """W 8192 noise tiles with most samples flagged (a threshold of at most
    one MAD): the tile's pool of flagged 4-sample parts runs several rounds
    of its list (up to 2048 parts against 256 per round); equal to the
    oracle in the one-class and fused launches."""
    specs = [synth.StreamSpec(8192 * 3 + 211, 8192, k, rfi.NOISE, 400.0, 0.01, 32, 32, "i16"),
             synth.StreamSpec(8192 * 2, 8192, k, rfi.NOISE, 30.0, 0.0, 1, 1, "i16")]
    x = synth.gen_packed(specs, seed=int(k * 10) + 3, tag=24)
    for sched in ("split", "split_persist", "fused"):
        y, st = gpu_run(x, specs, 14, gpu, schedule=sched)
        check_against_oracle(x, specs, 14, y, st)


@pytest.mark.parametrize("mode", MODES)
def test_degenerate(gpu, mode):
    rng = np.random.default_rng(2)
    W = 8192
    streams = [np.full(W * 2, -300, np.int16),
               rng.choice([-32768, 32767], W * 2).astype(np.int16),
               np.where(rng.random(W * 2) < 0.5, -20000, 20000).astype(np.int16),
               rng.integers(-32768, 32768, W * 2 + 1).astype(np.int16),
               np.zeros(0, np.int16),
               np.array([-32768, 32767], np.int16)]
    streams[0][17] = 32767
    x = synth.pack([torch.as_tensor(s) for s in streams])
    specs = [synth.StreamSpec(len(s), W, 3.0, mode, 1, 0, 1, 1, "i16") for s in streams]
    y, st = gpu_run(x, specs, 3, gpu)
    check_against_oracle(x, specs, 3, y, st)


def _band_and_radix_windows(rng, n_each=3):
    """W 8192 windows of every kind the tile's two selection paths see: the
    full-resolution band around the estimated median (narrow and moderate
    spreads, bursts, a median far from zero) and the radix fallback (median
    or MAD outside the band: wide spreads, uniform, bimodal, a level step
    inside the window)."""
    W = 8192
    g = lambda mu, sd: np.clip(np.round(rng.normal(mu, sd, W)), -32768, 32767)
    out = []
    for _ in range(n_each):
        out.append(g(int(rng.integers(-30000, 30000)), 400))        # band
        out.append(g(0, float(rng.choice([1, 30, 2000]))))          # band
        t = g(0, 400)
        idx = rng.random(W) < 0.01
        t[idx] = np.clip(50 * 400 * rng.standard_t(2, int(idx.sum())), -32768, 32767)
        out.append(t)                                               # band, Student-t bursts
        out.append(g(0, float(rng.choice([3000, 12000]))))          # MAD past the band
        out.append(rng.integers(-32768, 32768, W))                  # uniform
        out.append(np.where(rng.random(W) < 0.5, -25000, 25000))    # bimodal
        t = g(0, 400)
        t[int(rng.integers(1, 4)) * 2048:] += int(rng.integers(5000, 20000))
        out.append(np.clip(t, -32768, 32767))                       # level step
        out.append(g(32700, 50))                                    # band clipped at the top
        out.append(g(-32700, 50))                                   # band clipped at the bottom
    return np.concatenate(out).astype(np.int16)


@pytest.mark.parametrize("mode", MODES)
def test_w8192_band_and_radix_paths(gpu, mode):
    """Every window kind through the W 8192 tile, both selection paths,
    equal to the oracle in samples and statistics."""
    rng = np.random.default_rng(31 + mode)
    s = _band_and_radix_windows(rng)
    x = synth.pack([torch.as_tensor(s), torch.as_tensor(s[::-1].copy())])
    specs = [synth.StreamSpec(len(s), 8192, k, mode, 1, 0, 1, 1, "i16") for k in (3.0, 2.0)]
    for sched in ("split", "fused"):
        y, st = gpu_run(x, specs, 12, gpu, schedule=sched)
        check_against_oracle(x, specs, 12, y, st)


def test_all_schedules(gpu):
    specs = [synth.StreamSpec(8192 * 3 + 100, 8192, 3.0, rfi.NOISE, 400.0, 0.01, 32, 32, "i16"),
             synth.StreamSpec(9000, 2000, 2.5, rfi.CLIP, 200.0, 0.01, 32, 32, "i16")]
    x = synth.gen_packed(specs, seed=3, tag=22)
    ref = None
    for sched in ("split", "split_persist", "fused", "fused_persist", "per_stream", "split_concurrent", "fused_concurrent",
                  "one_launch", "one_launch_persist"):
        for graph in (False, True):
            y, st = gpu_run(x, specs, 1, gpu, schedule=sched, graph=graph, repeat=2)
            if ref is None:
                ref = check_against_oracle(x, specs, 1, y, st)
            else:
                L, W, _, _ = unpack(specs)
                so, _, _, _ = rfi.layout(L, W)
                for o, n in zip(so, L):
                    assert np.array_equal(y[o:o + n], ref[0][o:o + n]), (sched, graph)
                assert np.array_equal(st, ref[1])


def test_full_size_sampled(gpu):
    """60 x 2^23 int16, sigma 400, Student-t bursts, W 8192, k 3, noise."""
    rng = np.random.default_rng(8)
    specs = synth.int16_path()
    x = synth.gen_packed(specs, seed=0, tag=30, device=gpu)
    L, W, K, M = unpack(specs)
    y, st = rfi.mad_filter(x, L, W, K, M, seed=99)
    torch.cuda.synchronize()
    so, wo, nw, _ = rfi.layout(L, W)
    stn = rfi.stats_numpy(st)
    picks = rng.integers(0, nw, 80)
    picks[:2] = [0, nw - 1]
    for p in picks:
        s = int(np.searchsorted(wo, p, side="right") - 1)
        w = int(p - wo[s])
        a = int(so[s]) + w * 8192
        xs = x[a:a + 8192].cpu().numpy()
        yo, sto = oracle.window(xs, K[s], M[s], abs_start=w * 8192, stream=s, seed=99)
        assert np.array_equal(y[a:a + 8192].cpu().numpy(), yo), (s, w)
        assert stn[p] == sto, (s, w)
