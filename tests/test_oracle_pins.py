"""Pins of the CPU oracle against things other than itself (CPU only).

Each test ties part of the oracle to a fixed point outside it: hand-worked
windows, counting (brute-force) definitions, library routines that reduce to
the same quantity, closed-form statistics, invariants of the method, and
published known-answer vectors.  Paper: Sec. II-D, Eqs. (1)-(2).
"""
import itertools
import json
import math
import os
from statistics import NormalDist

import numpy as np
import pytest
import torch

import oracle
from paper_1710_08576_amd import synth

from _expect import rounded_gaussian_pmf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- hand-worked
@pytest.mark.parametrize("case", _load("hand_examples.json")["windows"], ids=lambda c: c["name"])
def test_hand_worked_window(case):
    x = np.array(case["x"], dtype=np.int8)
    y, st = oracle.window(x, case["k"], case["mode"])
    assert y.tolist() == case["y"]
    assert int(st["median"]) == case["median"]
    assert int(st["mad"]) == case["mad"]
    assert int(st["n_flagged"]) == case["n_flagged"]
    assert float(st["threshold"]) == case["threshold"]


@pytest.mark.parametrize("case", _load("hand_examples.json")["streams"], ids=lambda c: c["name"])
def test_hand_worked_stream(case):
    x = np.array(case["x"], dtype=np.int8)
    y, st = oracle.filter_batch(x, [len(x)], [case["window"]], case["k"], case["mode"])
    assert y.tolist() == case["y"]
    assert st["median"].tolist() == case["median"]
    assert st["mad"].tolist() == case["mad"]
    assert st["n_flagged"].tolist() == case["n_flagged"]


# ---------------------------------------------------------------- brute force
def _count_median(x):
    """Smallest v with #{x <= v} >= r + 1, r = floor((N-1)/2)."""
    r = (len(x) - 1) // 2
    for v in range(-32768, 32768):
        if np.count_nonzero(x <= v) >= r + 1:
            return v
    raise AssertionError


def _count_mad(x, m):
    """Smallest d with #{|x - m| <= d} >= r + 1."""
    r = (len(x) - 1) // 2
    d = np.abs(x.astype(np.int64) - m)
    for v in range(0, 65536):
        if np.count_nonzero(d <= v) >= r + 1:
            return v
    raise AssertionError


def _batch_windows(windows, k=3.0, mode=oracle.CLIP, dtype=np.int8):
    """Run each window as its own stream in one oracle call."""
    lengths = [len(w) for w in windows]
    so, _, _ = oracle.layout(lengths, lengths)
    total = int(so[-1]) + synth.align_up(lengths[-1])
    x = np.zeros(total, dtype=dtype)
    for o, w in zip(so, windows):
        x[o:o + len(w)] = w
    y, st = oracle.filter_batch(x, lengths, lengths, k, mode)
    return [y[o:o + len(w)] for o, w in zip(so, windows)], st


def test_counting_definition_exhaustive_small():
    alphabet = [-128, -1, 0, 1, 2, 127]
    wins = [np.array(t, dtype=np.int8)
            for n in (1, 2, 3) for t in itertools.product(alphabet, repeat=n)]
    _, st = _batch_windows(wins)
    for w, s in zip(wins, st):
        m = _count_median(w.astype(np.int64))
        assert s["median"] == m
        assert s["mad"] == _count_mad(w, m)


def test_counting_definition_random_int8():
    rng = np.random.default_rng(1)
    wins = []
    for _ in range(3000):
        n = int(rng.integers(1, 65))
        kind = rng.integers(0, 3)
        if kind == 0:
            w = rng.integers(-128, 128, n)
        elif kind == 1:
            w = np.clip(np.rint(rng.normal(0, 3, n)), -128, 127)
        else:
            w = rng.choice([-128, 127, 0, 5], n)
        wins.append(w.astype(np.int8))
    _, st = _batch_windows(wins)
    for w, s in zip(wins, st):
        x = w.astype(np.int64)
        r = (len(x) - 1) // 2
        # vectorised counting definition over all 256 candidate values
        v = np.arange(-128, 128)
        m = int(v[np.argmax((x[None, :] <= v[:, None]).sum(1) >= r + 1)])
        d = np.abs(x - m)
        dv = np.arange(0, 256)
        D = int(dv[np.argmax((d[None, :] <= dv[:, None]).sum(1) >= r + 1)])
        assert (s["median"], s["mad"]) == (m, D)


def test_counting_definition_1e5_windows():
    """10^5 random int8 windows of N = 1..64: the oracle's median and MAD
    equal the counting definitions (smallest v with #{x <= v} >= r + 1,
    smallest d with #{|x - m| <= d} >= r + 1), evaluated vectorised per N."""
    rng = np.random.default_rng(21)
    n_of = rng.integers(1, 65, 100_000)
    wins = []
    for n in n_of:
        kind = rng.integers(0, 3)
        if kind == 0:
            w = rng.integers(-128, 128, n)
        elif kind == 1:
            w = np.clip(np.rint(rng.normal(0, rng.uniform(0.5, 20), n)), -128, 127)
        else:
            w = rng.choice([-128, 127, 0, 5, -5], n)
        wins.append(w.astype(np.int8))
    _, st = _batch_windows(wins)
    got_m, got_d = np.asarray(st["median"]), np.asarray(st["mad"])
    for n in range(1, 65):
        idx = np.nonzero(n_of == n)[0]
        X = np.stack([wins[i] for i in idx]).astype(np.int64)  # (c, n)
        r = (n - 1) // 2
        rows = np.arange(len(idx))[:, None]
        h = np.zeros((len(idx), 256), np.int64)
        np.add.at(h, (np.broadcast_to(rows, X.shape), X + 128), 1)
        m = np.argmax(np.cumsum(h, 1) >= r + 1, 1) - 128
        hd = np.zeros((len(idx), 256), np.int64)
        np.add.at(hd, (np.broadcast_to(rows, X.shape), np.abs(X - m[:, None])), 1)
        D = np.argmax(np.cumsum(hd, 1) >= r + 1, 1)
        assert np.array_equal(got_m[idx], m), n
        assert np.array_equal(got_d[idx], D), n


def test_counting_definition_random_int16():
    rng = np.random.default_rng(2)
    wins = [rng.integers(-32768, 32768, int(rng.integers(1, 40))).astype(np.int16)
            for _ in range(200)]
    wins += [np.clip(np.rint(rng.normal(0, 400, 33)), -32768, 32767).astype(np.int16)
             for _ in range(100)]
    _, st = _batch_windows(wins, dtype=np.int16)
    for w, s in zip(wins, st):
        x = np.sort(w.astype(np.int64))
        r = (len(x) - 1) // 2
        # the counting definition is satisfied exactly at the reported values
        m = int(s["median"])
        assert np.count_nonzero(x <= m) >= r + 1 and np.count_nonzero(x <= m - 1) < r + 1
        D = int(s["mad"])
        d = np.abs(x - m)
        assert np.count_nonzero(d <= D) >= r + 1
        assert D == 0 or np.count_nonzero(d <= D - 1) < r + 1


# ---------------------------------------------------------------- libraries
def test_torch_median_is_lower_median():
    """torch.median (CPU) returns the lower of the two middle values."""
    rng = np.random.default_rng(3)
    wins = [rng.integers(-128, 128, int(rng.integers(1, 200))).astype(np.int8)
            for _ in range(500)]
    _, st = _batch_windows(wins)
    for w, s in zip(wins, st):
        t = torch.from_numpy(w.astype(np.int64))
        m = int(torch.median(t))
        D = int(torch.median((t - m).abs()))
        assert (s["median"], s["mad"]) == (m, D)


def test_numpy_scipy_odd_windows():
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(4)
    wins = [np.clip(np.rint(rng.normal(0, 12, 2 * int(rng.integers(0, 300)) + 1)),
                    -128, 127).astype(np.int8) for _ in range(300)]
    _, st = _batch_windows(wins)
    for w, s in zip(wins, st):
        x = w.astype(np.float64)
        assert s["median"] == np.median(x)
        assert s["mad"] == scipy_stats.median_abs_deviation(x, scale=1.0)


# ---------------------------------------------------------------- threshold
def test_threshold_binary32_rounding():
    """t is two binary32 round-to-nearest products, 1.4826f*D then k*that,
    within two half-ulps of the real product k * 1.4826f * D."""
    rng = np.random.default_rng(5)
    Ds = list(range(0, 256)) + [int(v) for v in rng.integers(256, 32768, 200)]
    for D in Ds:
        k = np.float32(rng.uniform(0.0, 10.0))
        # window [0, D, D, -D, -D]: lower median 0, MAD D
        w = np.array([0, D, D, -D, -D], dtype=np.int16)
        _, st = oracle.window(w, float(k), oracle.CLIP)
        assert int(st["median"]) == 0 and int(st["mad"]) == D
        t = np.float32(st["threshold"])
        assert t == np.float32(k * np.float32(np.float32(1.4826) * np.float32(D)))
        exact = float(k) * float(np.float32(1.4826)) * D
        assert abs(float(t) - exact) <= 2 * float(np.spacing(np.float32(exact)))


def test_flag_strictness_at_integer_threshold():
    """Eq. (2) is read strictly: with D = 0, samples equal to m stay."""
    x = np.array([4, 4, 4, 4, 4, 9], dtype=np.int8)
    y, st = oracle.window(x, 3.0, oracle.ZERO)
    assert st["mad"] == 0 and st["n_flagged"] == 1 and y.tolist() == [4, 4, 4, 4, 4, 0]


# ---------------------------------------------------------------- invariants
def _rand_stream(rng, n, sigma=10.0, dtype=np.int8, lo=-128, hi=127):
    x = np.rint(rng.normal(0, sigma, n))
    idx = rng.integers(0, n, max(1, n // 50))
    x[idx] += rng.choice([-1, 1], len(idx)) * rng.integers(60, 128, len(idx))
    return np.clip(x, lo, hi).astype(dtype)


@pytest.mark.parametrize("W", [7, 64, 500, 4096])
def test_invariants(W):
    rng = np.random.default_rng(6 + W)
    L = 3 * W + W // 3 + 1
    x = _rand_stream(rng, L)
    outs = {m: oracle.filter_batch(x, [L], [W], 3.0, m) for m in (0, 1, 2)}
    y0, st0 = outs[0]
    for m in (1, 2):
        # I2: flags and stats do not depend on the mode
        assert np.array_equal(outs[m][1], st0)
    nw = len(st0)
    for w in range(nw):
        a, b = w * W, min(L, (w + 1) * W)
        xs = x[a:b].astype(np.int64)
        med, T = int(st0["median"][w]), int(math.floor(st0["threshold"][w]))
        flag = np.abs(xs - med) > T
        for m in (0, 1, 2):
            ys = outs[m][0][a:b].astype(np.int64)
            # I1: unflagged samples unchanged in every mode
            assert np.array_equal(ys[~flag], xs[~flag])
        # I3: ZERO changes exactly the flagged non-zero samples
        assert np.count_nonzero(outs[0][0][a:b] != x[a:b]) == np.count_nonzero(flag & (xs != 0))
        assert st0["n_flagged"][w] == np.count_nonzero(flag)
        # I4: CLIP output lies within [m - T, m + T] for flagged samples
        yc = outs[1][0][a:b].astype(np.int64)
        assert np.all(yc[flag] >= max(med - T, -128)) and np.all(yc[flag] <= min(med + T, 127))


def test_raising_k_never_raises_flags():
    rng = np.random.default_rng(7)
    x = _rand_stream(rng, 8192)
    prev = None
    for k in (0.0, 0.5, 1.0, 2.0, 2.5, 3.0, 4.0, 8.0, 100.0):
        _, st = oracle.filter_batch(x, [len(x)], [1024], k, 0)
        if prev is not None:
            assert np.all(st["n_flagged"] <= prev)
        prev = st["n_flagged"]


def test_translation_and_permutation():
    rng = np.random.default_rng(8)
    x = np.clip(np.rint(rng.normal(0, 8, 4096)), -90, 90).astype(np.int8)
    _, st = oracle.window(x, 3.0, 0)
    # I6: translation by c moves m, leaves D and flags
    for c in (-30, 17):
        _, st2 = oracle.window((x.astype(np.int16) + c).astype(np.int8), 3.0, 0)
        assert st2["median"] == st["median"] + c and st2["mad"] == st["mad"]
        assert st2["n_flagged"] == st["n_flagged"]
    # I7: permutation leaves m, D, n_flagged
    _, st3 = oracle.window(rng.permutation(x), 3.0, 0)
    assert (st3["median"], st3["mad"], st3["n_flagged"]) == (st["median"], st["mad"], st["n_flagged"])
    # I8: negation of an odd window with no -128 negates m, keeps D
    xo = x[:4095]
    _, a = oracle.window(xo, 3.0, 0)
    _, b = oracle.window((-xo.astype(np.int16)).astype(np.int8), 3.0, 0)
    assert b["median"] == -a["median"] and b["mad"] == a["mad"]


def test_block_split_invariance():
    """I9: splitting a stream at window multiples gives identical output,
    given the absolute sample index for the noise key."""
    rng = np.random.default_rng(9)
    W, L = 512, 512 * 9 + 100
    x = _rand_stream(rng, L)
    y, st = oracle.filter_batch(x, [L], [W], 3.0, oracle.NOISE, seed=42)
    for w in range(len(st)):
        a, b = w * W, min(L, (w + 1) * W)
        yw, sw = oracle.window(x[a:b], 3.0, oracle.NOISE, abs_start=a, stream=0, seed=42)
        assert np.array_equal(yw, y[a:b]) and sw == st[w]


# ---------------------------------------------------------------- statistics
def test_int16_gaussian_closed_forms():
    """Pure Gaussian int16, sigma 400: MAD/sigma ~ 0.6745, flag rate ~ 2 Phi(-3)."""
    g = torch.Generator().manual_seed(10)
    x = torch.clamp(torch.round(torch.randn(1 << 21, generator=g) * 400), -32768, 32767)
    x = x.to(torch.int16).numpy()
    _, st = oracle.filter_batch(x, [len(x)], [8192], 3.0, 0)
    mad_ratio = st["mad"].mean() / 400.0
    assert abs(mad_ratio - 0.6745) < 0.004
    frac = st["n_flagged"].sum() / len(x)
    assert abs(frac - 2 * NormalDist().cdf(-3)) < 0.0004


@pytest.mark.parametrize("sigma", [6.0, 10.0])
def test_int8_discrete_expectations(sigma):
    """int8 quantisation moves MAD and the flag rate off the continuous values;
    compare with the exact discrete expectation from the rounded-Gaussian pmf."""
    pmf = np.array(rounded_gaussian_pmf(sigma, -128, 127))
    vals = np.arange(-128, 128)
    # population median is 0 by symmetry; population MAD: smallest d with P(|X|<=d) >= 1/2
    cum = np.array([pmf[np.abs(vals) <= d].sum() for d in range(128)])
    D_pop = int(np.argmax(cum >= 0.5))
    t = np.float32(3.0) * (np.float32(1.4826) * np.float32(D_pop))
    T = int(math.floor(t))
    p_flag = pmf[np.abs(vals) > T].sum()
    g = torch.Generator().manual_seed(11)
    x = torch.clamp(torch.round(torch.randn(1 << 22, generator=g) * sigma), -128, 127)
    x = x.to(torch.int8).numpy()
    _, st = oracle.filter_batch(x, [len(x)], [16384], 3.0, 0)
    assert np.all(st["median"] == 0)
    assert np.mean(st["mad"] == D_pop) > 0.95
    frac = st["n_flagged"].sum() / len(x)
    assert abs(frac - p_flag) < 0.15 * p_flag + 2e-4


def test_noise_statistics():
    """Noise replacements: zero mean, spread ~ sigma_hat, and no correlation
    between neighbouring samples that share a Philox block."""
    g = torch.Generator().manual_seed(12)
    L = 1 << 20
    x = torch.clamp(torch.round(torch.randn(L, generator=g) * 20), -128, 127).to(torch.int8).numpy()
    y, st = oracle.filter_batch(x, [L], [4096], 0.0, oracle.NOISE, seed=5)
    # with k = 0 every sample != m is replaced by m + q; collect q
    med = np.repeat(st["median"], 4096)[:L]
    q = y.astype(np.int64) - med
    flag = x.astype(np.int64) != med
    qs = q[flag]
    sig = np.repeat(1.4826 * st["mad"], 4096)[:L][flag]
    z = qs / sig
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.02
    # correlation of q at lags inside and across 4-sample Philox blocks
    qf = np.where(flag, q, 0).astype(np.float64)
    for lag in (1, 2, 3, 4, 15):
        a, b = qf[:-lag], qf[lag:]
        both = flag[:-lag] & flag[lag:]
        c = np.corrcoef(a[both], b[both])[0, 1]
        assert abs(c) < 0.01, (lag, c)


def test_noise_distribution_chi2():
    """With k = 0 every sample != m takes m + q; for windows sharing (m, D)
    the q values must follow the distribution that uniform 12-bit indices
    induce through the Q8 table and the scale s (chi-square, p > 1e-4)."""
    W = 64
    base = np.array([-4] * 8 + [-2] * 16 + [0] * 9 + [2] * 16 + [4] * 15, dtype=np.int8)
    rng = np.random.default_rng(5)
    n_win = 1 << 14
    x = np.concatenate([rng.permutation(base) for _ in range(n_win)])
    y, st = oracle.filter_batch(x, [len(x)], [W], 0.0, oracle.NOISE, seed=9)
    assert np.all(st["median"] == 0) and np.all(st["mad"] == 2)
    sq8 = int(np.float32(np.float32(np.float32(1.4826) * np.float32(2)) * np.float32(256.0)))
    G = oracle.q8_table().astype(np.int64)
    qv = (sq8 * G + 32768) // 65536
    vals, cnt = np.unique(qv, return_counts=True)
    p = cnt / 4096.0
    q = y.astype(np.int64)[x != 0]
    obs = np.array([(q == v).sum() for v in vals])
    assert obs.sum() == len(q)  # every q is a table value
    exp = p * len(q)
    keep = exp >= 5
    chi2 = (((obs - exp) ** 2) / exp)[keep].sum() + \
        ((obs[~keep].sum() - exp[~keep].sum()) ** 2 / max(exp[~keep].sum(), 1e-9))
    df = int(keep.sum())  # kept cells + pooled tail - 1
    assert chi2 < df + 6 * math.sqrt(2 * df), (chi2, df)


# ---------------------------------------------------------------- noise parts
def test_q8_table_matches_normaldist():
    G = oracle.q8_table()
    ref = np.array([round(256 * NormalDist().inv_cdf((u + 0.5) / 4096)) for u in range(4096)])
    assert np.array_equal(G, ref)
    assert np.array_equal(G, -G[::-1])
    assert np.all(np.diff(G) >= 0) and G.max() == 939


def test_philox_known_answer():
    for v in _load("philox4x64_10_kat.json")["vectors"]:
        out = oracle.philox4x64_10([int(c, 16) for c in v["ctr"]], [int(c, 16) for c in v["key"]])
        assert out == [int(c, 16) for c in v["out"]]


def test_philox_matches_numpy():
    rng = np.random.default_rng(13)
    for _ in range(50):
        c = int(rng.integers(1, 2**62))
        key = [int(rng.integers(0, 2**63)), int(rng.integers(0, 2**32))]
        bg = np.random.Philox(counter=c - 1, key=np.array(key, dtype=np.uint64))
        assert oracle.philox4x64_10([c, 0, 0, 0], key) == [int(v) for v in bg.random_raw(4)]


def test_noise_value_from_library_parts():
    """A flagged sample's noise, rebuilt from numpy's Philox and NormalDist."""
    x = np.concatenate([np.arange(-20, 21), [100, 101, -100, 127, -128], np.zeros(15)])
    x = x.astype(np.int8)
    seed, stream, a = 77, 3, 4096 * 5
    y, st = oracle.window(x, 1.0, oracle.NOISE, abs_start=a, stream=stream, seed=seed)
    m, D = int(st["median"]), int(st["mad"])
    assert D > 0
    sig = np.float32(np.float32(1.4826) * np.float32(D))
    sq8 = int(np.float32(sig * np.float32(256.0)))
    T = math.floor(float(st["threshold"]))
    n_checked = 0
    for i, v in enumerate(x.astype(np.int64)):
        if abs(v - m) <= T:
            assert y[i] == v
            continue
        j = a + i
        bg = np.random.Philox(counter=(j >> 2) - 1, key=np.array([seed, stream], dtype=np.uint64))
        word = int(bg.random_raw(4)[j & 3])
        u = word >> 52
        G = round(256 * NormalDist().inv_cdf((u + 0.5) / 4096))
        q = (sq8 * G + 32768) // 65536
        assert y[i] == max(-128, min(127, m + q))
        n_checked += 1
    assert n_checked >= 5


def test_layout():
    so, wo, total = oracle.layout([10, 0, 64, 65], [4, 3, 64, 10])
    assert so.tolist() == [0, 64, 64, 128] and wo.tolist() == [0, 3, 3, 4] and total == 11
