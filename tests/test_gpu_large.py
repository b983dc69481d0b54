"""Maximum sizes: a stream longer than 2^31 samples (byte offsets past 2^31
for int8 and past 2^32 for int16), checked window by window against the
oracle around the 32-bit boundaries and at the stream's end."""
import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

pytestmark = pytest.mark.gpu

N_LONG = (1 << 31) + 3 * 8192 + 100


def _check_windows(x, y, st, lengths, W, k, mode, seed, windows):
    so, wo, _, _ = rfi.layout(lengths, [W] * len(lengths))
    stn = rfi.stats_numpy(st)
    s = len(lengths) - 1
    for w in windows:
        a = int(so[s]) + w * W
        n = min(W, lengths[s] - w * W)
        xs = x[a:a + n].cpu().numpy()
        yo, sto = oracle.window(xs, k, mode, abs_start=w * W, stream=s, seed=seed)
        assert np.array_equal(y[a:a + n].cpu().numpy(), yo), (W, mode, w)
        assert stn[int(wo[s]) + w] == sto, (W, mode, w)


@pytest.mark.parametrize("W,mode", [(4096, rfi.NOISE), (5000, rfi.CLIP)])
def test_int8_stream_past_2_31(gpu, W, mode):
    lengths = [5, N_LONG]
    total = rfi.layout(lengths, [W, W])[3]
    g = torch.Generator(device=gpu)
    g.manual_seed(11)
    x = torch.randint(-128, 128, (total,), generator=g, dtype=torch.int8, device=gpu)
    # a stretch of Gaussian-like samples with a burst around the 2^31 boundary
    b = (1 << 31) - 20000
    x[b:b + 40000] = torch.clamp(torch.randn(40000, generator=g, device=gpu) * 12, -128, 127).to(torch.int8)
    x[b + 19000:b + 21000] = 120
    y, st = rfi.mad_filter(x, lengths, [W, W], [3.0, 3.0], [mode, mode], seed=77)
    torch.cuda.synchronize()
    nw = (N_LONG + W - 1) // W
    edge = (1 << 31) // W
    _check_windows(x, y, st, lengths, W, 3.0, mode, 77,
                   [0, 1, edge - 2, edge - 1, edge, edge + 1, nw - 2, nw - 1])
    del x, y, st
    torch.cuda.empty_cache()


def test_int16_stream_past_2_32_bytes(gpu):
    W, mode = 8192, rfi.NOISE
    lengths = [3, N_LONG]
    total = rfi.layout(lengths, [W, W])[3]
    g = torch.Generator(device=gpu)
    g.manual_seed(12)
    x = (torch.randn(total, generator=g, device=gpu) * 400).round().clamp(-32768, 32767).to(torch.int16)
    b = (1 << 31) - 30000
    x[b + 25000:b + 26000] = -32768
    y, st = rfi.mad_filter(x, lengths, [W, W], [3.0, 3.0], [mode, mode], seed=78)
    torch.cuda.synchronize()
    nw = (N_LONG + W - 1) // W
    edge = (1 << 31) // W
    _check_windows(x, y, st, lengths, W, 3.0, mode, 78,
                   [0, edge - 1, edge, edge + 1, nw - 2, nw - 1])
    del x, y, st
    torch.cuda.empty_cache()
