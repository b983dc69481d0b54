"""Pins of the median-of-MAD oracle (Eq. (3)), CPU only.

Reading: for window w the threshold uses the lower median of the MADs of
windows max(0, w-K+1) .. w of the same stream; the centre stays the window's
own median M(x).  Pinned by hand-worked streams, by its reduction to the
plain filter (K = 1, or every window with the same MAD), and by a numpy
evaluation of the definition on random streams.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1710_08576_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mom(x, W, K, k, mode, seed=0):
    y, st = oracle.mom_filter_batch(x, [len(x)], [W], k, mode, K, seed=seed)
    return y[:len(x)], st


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "mom_examples.json")))["streams"],
                         ids=lambda c: c["name"])
def test_hand_worked_streams(case):
    x = np.array(case["x"], dtype=np.int8)
    y, st = _mom(x, case["window"], case["mom_k"], case["k"], case["mode"])
    assert y.tolist() == case["y"]
    assert st["median"].tolist() == case["median"]
    assert st["mad"].tolist() == case["mad"]
    assert st["n_flagged"].tolist() == case["n_flagged"]
    assert st["threshold"].tolist() == case["threshold"]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_k1_is_the_plain_filter(mode):
    spec = synth.StreamSpec(50_000, 1000, 3.0, mode, 12.0, 0.01, 8, 300)
    x = synth.gen_stream(spec, 3, 7, 0).numpy()
    y1, s1 = _mom(x, 1000, 1, 3.0, mode, seed=4)
    y0, s0 = oracle.filter_batch(x, [len(x)], [1000], 3.0, mode, seed=4)
    assert np.array_equal(y1, y0[:len(x)])
    assert np.array_equal(s1, s0)


def test_equal_mads_give_the_plain_filter():
    """Every window a permutation of one pattern: all MADs equal, so any K
    gives the plain filter."""
    rng = np.random.default_rng(2)
    base = np.clip(np.rint(rng.normal(0, 9, 512)), -128, 127).astype(np.int8)
    base[:5] = [100, -100, 90, 127, -128]
    x = np.concatenate([rng.permutation(base) for _ in range(40)])
    y0, s0 = oracle.filter_batch(x, [len(x)], [512], 2.5, 1)
    for K in (2, 7, 40, 1000):
        y, s = _mom(x, 512, K, 2.5, 1)
        assert np.array_equal(y, y0[:len(x)]) and np.array_equal(s, s0)


@pytest.mark.parametrize("W,K", [(64, 5), (100, 16), (256, 3)])
def test_numpy_definition(W, K):
    """Median, MAD, the sliding lower median of MADs, the binary32 threshold
    and ZERO/CLIP replacement evaluated with numpy sorts."""
    rng = np.random.default_rng(W + K)
    L = W * 37 + W // 3
    sig = np.repeat(rng.uniform(2, 25, L // W + 1), W)[:L]  # MAD varies window to window
    x = np.clip(np.rint(rng.normal(0, 1, L) * sig), -128, 127)
    burst = rng.random(L) < 0.01
    x = np.where(burst, np.clip(x + rng.choice([-90, 90], L), -128, 127), x).astype(np.int8)
    for mode in (0, 1):
        y, st = _mom(x, W, K, 2.75, mode)
        nw = (L + W - 1) // W
        med, mad = [], []
        for w in range(nw):
            v = np.sort(x[w * W:(w + 1) * W].astype(np.int64))
            r = (len(v) - 1) // 2
            med.append(int(v[r]))
            mad.append(int(np.sort(np.abs(v - v[r]))[r]))
        for w in range(nw):
            win = np.sort(np.array(mad[max(0, w - K + 1):w + 1]))
            Dm = int(win[(len(win) - 1) // 2])
            t = np.float32(np.float32(2.75) * np.float32(np.float32(1.4826) * np.float32(Dm)))
            T = int(np.floor(t))
            xs = x[w * W:(w + 1) * W].astype(np.int64)
            flag = np.abs(xs - med[w]) > float(t)
            if mode == 0:
                exp = np.where(flag, 0, xs)
            else:
                exp = np.clip(xs, max(med[w] - T, -128), min(med[w] + T, 127))
            assert np.array_equal(y[w * W:(w + 1) * W], exp), (mode, w)
            assert st[w]["median"] == med[w] and st[w]["mad"] == mad[w]
            assert st[w]["n_flagged"] == flag.sum() and st[w]["threshold"] == t


def test_rejects_bad_k():
    with pytest.raises(ValueError):
        oracle.mom_filter_batch(np.zeros(8, np.int8), [8], [4], 3.0, 1, 0)
