"""Microbenchmark kernels: the HBM copy and the LDS histogram rate give
exact results (a copy; numpy's byte counts)."""
import numpy as np
import pytest
import torch

import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_copy_variants(gpu, variant):
    g = torch.Generator(device=gpu)
    g.manual_seed(variant)
    x = torch.randint(-128, 128, (16384 * 37,), generator=g, dtype=torch.int8, device=gpu)
    y = torch.zeros_like(x)
    _lib.ubench_copy(x, y, variant)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@pytest.mark.parametrize("replicas", [1, 2, 4, 8])
def test_lds_hist_counts(gpu, replicas):
    rng = np.random.default_rng(replicas)
    xn = np.concatenate([rng.integers(-128, 128, 16384 * 5),
                         np.clip(np.round(rng.normal(0, 6, 16384 * 3)), -128, 127)]).astype(np.int8)
    x = torch.from_numpy(xn).to(gpu)
    h = _lib.ubench_lds_hist(x, replicas)
    h = _lib.ubench_lds_hist(x, replicas, hist=h)  # accumulates
    torch.cuda.synchronize()
    want = 2 * np.bincount(xn.view(np.uint8), minlength=256)
    assert np.array_equal(h.cpu().numpy().astype(np.int64).sum(axis=0), want)


def test_lds_hist_errors(gpu):
    x = torch.zeros(16384, dtype=torch.int8, device=gpu)
    for r in (0, 3, 16):
        with pytest.raises(rfi.RfiError):
            _lib.ubench_lds_hist(x, r)
    with pytest.raises(rfi.RfiError):
        _lib.ubench_lds_hist(x[:1000], 4)
