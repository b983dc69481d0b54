"""Several outputs from one read: each output equals the single-output call
and the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

pytestmark = pytest.mark.gpu
SENT = 0x5A


def _specs():
    out = []
    for i, (W, L) in enumerate([(4096, 4096 * 33 + 77), (512, 512 * 100), (1000, 40_000),
                                (16384, 16384 * 4 + 5), (2048, 2048 * 40), (8192, 8192 * 6),
                                (1024, 1024 * 50 + 3), (300, 9_000)]):
        out.append(synth.StreamSpec(L, W, 3.0, 1, 5.0 + 2.0 * i, 0.015, 8, 400))
    return out


@pytest.mark.parametrize("n_out", [1, 2, 3])
def test_outputs_match_oracle(gpu, n_out):
    specs = _specs()
    L = [s.length for s in specs]
    W = [s.window for s in specs]
    x = synth.gen_packed(specs, 12, 51).numpy()
    ns = len(specs)
    rng = np.random.default_rng(n_out)
    ks = [np.float32(rng.uniform(2.0, 5.0, ns)) for _ in range(n_out)]
    modes = [np.array([(o + s) % 3 for s in range(ns)], np.int32) for o in range(n_out)]
    xd = torch.from_numpy(x.copy()).to(gpu)
    ys = [torch.full_like(xd, SENT) for _ in range(n_out)]
    ys, sts = rfi.mad_filter_multi(xd, L, W, ks, modes, seed=6, ys=ys)
    torch.cuda.synchronize()
    so = rfi.layout(L, W)[0]
    for o in range(n_out):
        yo, sto = oracle.filter_batch(x, L, W, ks[o], modes[o], seed=6)
        y = ys[o].cpu().numpy()
        for s, (off, n) in enumerate(zip(so, L)):
            assert np.array_equal(y[off:off + n], yo[off:off + n]), (o, s)
            assert np.all(y[off + n:off + synth.align_up(n)].view(np.uint8) == SENT)
        assert np.array_equal(rfi.stats_numpy(sts[o]), sto), o


def test_equals_single_calls(gpu):
    specs = synth.plain_scale(8, 1 << 20, 4096, rfi.CLIP)
    L = [s.length for s in specs]
    xd = synth.gen_packed(specs, 0, 3, device=gpu)
    ks = [[3.0] * 8, [2.5] * 8, [4.0] * 8]
    modes = [[0] * 8, [1] * 8, [2] * 8]
    ys, sts = rfi.mad_filter_multi(xd, L, [4096] * 8, ks, modes, seed=2)
    for o in range(3):
        y1, s1 = rfi.mad_filter(xd, L, [4096] * 8, ks[o], modes[o], seed=2)
        assert torch.equal(ys[o], y1)
        assert torch.equal(sts[o], s1)


def test_overlap_rejected(gpu):
    xd = torch.zeros(4096, dtype=torch.int8, device=gpu)
    y = torch.empty_like(xd)
    with pytest.raises(rfi.RfiError):
        rfi.mad_filter_multi(xd, [4096], [1024], [[3.0], [3.0]], [[1], [1]], ys=[y, y])
    with pytest.raises(rfi.RfiError):
        rfi.mad_filter_multi(xd, [4096], [1024], [[3.0]], [[1]], ys=[xd])
    with pytest.raises(rfi.RfiError):
        rfi.mad_filter_multi(xd, [4096], [1024], [[3.0]] * 4, [[1]] * 4)
