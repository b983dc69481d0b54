"""Pins of the oracle's improvement metric (Sec. III-A) and of the MAD
breakdown that motivates the median of MAD (Sec. II-D, Sec. III-B, the
emulator comparison).  CPU only."""
import numpy as np
import pytest

import oracle
from paper_1710_08576_amd import synth


# --------------------------------------------------------------- block power

def test_block_power_brute_force_int8_and_int16():
    rng = np.random.default_rng(5)
    for dt, lo, hi in ((np.int8, -128, 127), (np.int16, -32768, 32767)):
        lengths = [0, 1, 63, 64, 65, 1000]
        total = sum((L + 63) // 64 * 64 for L in lengths)
        x = rng.integers(lo, hi + 1, total).astype(dt)
        x[:5] = lo  # extremes inside the first blocks
        for block in (1, 7, 64, 300, 4096):
            got = oracle.block_power(x, lengths, block)
            want = []
            off = 0
            for L in lengths:
                vals = [int(v) for v in x[off:off + L]]
                for b in range(0, L, block):
                    want.append(sum(v * v for v in vals[b:b + block]))
                off += (L + 63) // 64 * 64
            assert got.tolist() == want


def test_block_power_closed_forms():
    # constant c: c^2 per sample; the short last block holds L % block samples
    x = np.full(1000, -7, dtype=np.int8)
    assert oracle.block_power(x, [1000], 300).tolist() == [49 * 300] * 3 + [49 * 100]
    # ramp 0..n-1 (int16): sum of squares n (n - 1) (2n - 1) / 6
    n = 20000
    r = np.arange(n, dtype=np.int64)
    x16 = np.where(r < 32768, r, 0).astype(np.int16)
    assert int(oracle.block_power(x16, [n], n)[0]) == (n - 1) * n * (2 * n - 1) // 6
    # the most negative int16 squared is 2^30 (no 16- or 32-bit wrap)
    big = np.full(8, -32768, dtype=np.int16)
    assert oracle.block_power(big, [8], 8).tolist() == [8 << 30]


# --------------------------------------------------------- the ratio S, metric

def test_s_ratio_two_level_closed_form():
    # a series alternating a, b: mean (a + b) / 2, RMS deviation |a - b| / 2,
    # so S = |a - b| / (a + b) (worked by hand, not from the code)
    for a, b, want in ((10, 30, 0.5), (5, 6, 1 / 11), (1000, 1, 999 / 1001)):
        assert oracle.s_ratio([a, b] * 8, 16) == pytest.approx(want, rel=1e-15)
    # averaging over segments: two segments with ratios 0.5 and 0.1
    s = oracle.s_ratio([10, 30] * 4 + [18, 22] * 4, 8)
    assert s == pytest.approx(0.3, rel=1e-15)
    # trailing values beyond the last whole segment are ignored
    assert oracle.s_ratio([10, 30] * 4 + [1e9], 8) == pytest.approx(0.5, rel=1e-15)
    assert np.isnan(oracle.s_ratio([1, 2, 3], 4))
    # no deviation: S = 0; no deviation and zero mean: 0 / 0
    assert oracle.s_ratio([5, 5, 5, 5], 4) == 0.0
    assert np.isnan(oracle.s_ratio([0, 0, 0, 0], 4))
    # a steadier series has the smaller S
    assert oracle.s_ratio([19, 21] * 8, 16) < oracle.s_ratio([10, 30] * 8, 16)


def test_s_ratio_gaussian_power():
    # P = sum of N squared N(0, sigma^2) samples: mean N sigma^2, standard
    # deviation sigma^2 sqrt(2N), so S = sqrt(2 / N) (rounding to integers
    # moves it by well under 1 % at sigma 10).
    N, nb = 4096, 1024
    g = np.random.default_rng(11)
    x = np.clip(np.round(g.normal(0, 10.0, N * nb)), -128, 127).astype(np.int8)
    p = oracle.block_power(x, [N * nb], N)
    s = oracle.s_ratio(p, 256)
    assert s == pytest.approx(np.sqrt(2 / N), rel=0.08)


def test_improvement_hand_example_and_invariances():
    # worked by hand: S_U = 20 / 40 = 0.5, S_F = 4 / 40 = 0.1, and the printed
    # 10 log10(S_U / S_F) = 10 log10 5 = +6.9897 dB: the steadier filtered
    # power scores a positive improvement.
    L, block = 16 * 5, 5
    pu = np.array([10, 30] * 8, dtype=np.int64)
    pf = np.array([18, 22] * 8, dtype=np.int64)
    r = oracle.improvement(pu, pf, [L], block, 16)[0]
    assert r[0] == pytest.approx(0.5, rel=1e-15) and r[1] == pytest.approx(0.1, rel=1e-15)
    assert r[2] == pytest.approx(6.989700043360188, abs=1e-12)
    # swapping the two inputs flips the sign
    assert oracle.improvement(pf, pu, [L], block, 16)[0][2] == pytest.approx(-6.989700043360188, abs=1e-12)
    # identical series: 0 dB; a constant gain on the filtered power: 0 dB
    assert oracle.improvement(pu, pu, [L], block, 16)[0][2] == 0.0
    assert oracle.improvement(pu, 4 * pu, [L], block, 16)[0][2] == pytest.approx(0.0, abs=1e-12)
    # the short last block of a stream is not used
    pu2 = np.concatenate([pu, [10 ** 9]])
    pf2 = np.concatenate([pf, [1]])
    r2 = oracle.improvement(pu2, pf2, [L + 3], block, 16)[0]
    assert r2.tolist() == r.tolist()
    # a stream with no whole segment: NaN throughout
    r3 = oracle.improvement(pu[:10], pf[:10], [50], block, 16)[0]
    assert np.all(np.isnan(r3))


def test_replacement_ranking_on_synthetic_bursts():
    # Sec. III-B, comparison of replacement options: zero and digital noise
    # improve the integrated power about equally, clipping at the threshold
    # much less; all three improve on the unfiltered signal.
    ns, L, block = 2, 1 << 22, 1 << 16
    specs = synth.plain_scale(ns, L, 4096, synth.ZERO)
    x = synth.gen_packed(specs, 0, 100).numpy()
    lengths = [s.length for s in specs]
    pu = oracle.block_power(x, lengths, block)
    imp = {}
    for name, m in (("zero", 0), ("clip", 1), ("noise", 2)):
        y, _ = oracle.filter_batch(x, lengths, [4096] * ns, 3.0, m, n_threads=4)
        imp[name] = oracle.improvement(pu, oracle.block_power(y, lengths, block), lengths, block, 16)[:, 2]
    for s in range(ns):
        assert imp["clip"][s] > 1.0
        assert imp["zero"][s] > imp["clip"][s] + 3.0
        assert imp["noise"][s] > imp["clip"][s] + 3.0
        assert abs(imp["zero"][s] - imp["noise"][s]) < 3.0


# ---------------------------------------------------- breakdown of the MAD

def _ideal_detection(x, mask, k=3.0):
    # a threshold detector that knows the burst-free statistics exactly
    clean = np.sort(x[~mask].astype(np.int64))
    m = clean[(len(clean) - 1) // 2]
    d = np.sort(np.abs(clean - m))[(len(clean) - 1) // 2]
    t = k * 1.4826 * d
    return float((np.abs(x[mask].astype(np.int64) - m) > t).mean())


@pytest.mark.parametrize("on", [2048, 8192, 51200])
def test_mad_misses_long_bursts_median_of_mad_does_not(on):
    # Sec. III-B: with windows of 16384 samples the MAD misses emulator
    # bursts lasting beyond ~10 us (8192 samples at 800 Msample/s, half a
    # window), while the median of MAD catches all of them.
    # the first burst starts after the 256-window history has filled
    L, period, phase = 1 << 22, 1 << 20, 256 * 4096 + 1000
    x = synth.gen_emulator_stream(L, 10.0, on, period, phase, 15.0, 0, 0).numpy()
    mask = synth.emulator_mask(L, on, period, phase).numpy()
    ideal = _ideal_detection(x, mask)
    y, _ = oracle.filter_batch(x, [L], [16384], 3.0, oracle.CLIP, n_threads=4)
    det_mad = float((y != x)[mask].mean())  # clip changes exactly the flagged samples
    y, _ = oracle.mom_filter_batch(x, [L], [4096], 3.0, oracle.CLIP, 256, n_threads=4)
    det_mom = float((y != x)[mask].mean())
    assert abs(det_mom - ideal) < 0.03
    if on <= 2048:
        assert det_mad > 0.9 * ideal
    elif on <= 8192:
        assert 0.2 * ideal < det_mad < 0.8 * ideal
    else:
        assert det_mad < 0.15 * ideal
