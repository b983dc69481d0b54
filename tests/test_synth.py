"""The synthetic inputs follow the recipe stated for them: seeded and
reproducible, the configured spreads, burst fractions and emulator timing."""
import numpy as np
import torch

from paper_1710_08576_amd import synth


def test_seeded_and_reproducible():
    specs = synth.plain_scale(3, 1 << 16, 4096, synth.CLIP)
    a = synth.gen_packed(specs, 0, 5)
    b = synth.gen_packed(specs, 0, 5)
    c = synth.gen_packed(specs, 1, 5)
    assert torch.equal(a, b) and not torch.equal(a, c)


def test_plain_scale_parameters():
    specs = synth.plain_scale()
    assert len(specs) == 60 and all(s.length == 1 << 24 and s.k == 3.0 for s in specs)
    assert all(6.0 <= s.sigma <= 20.0 and 0.001 <= s.frac <= 0.02 for s in specs)
    assert all(s.burst_lo == 8 and s.burst_hi == 512 for s in specs)


def test_gaussian_part_and_burst_fraction():
    L = 1 << 21
    spec = synth.StreamSpec(L, 4096, 3.0, synth.CLIP, 10.0, 0.01, 32, 32)
    x = synth.gen_stream(spec, 3, 0, 0).numpy().astype(np.int64)
    big = np.abs(x) >= 60  # burst magnitudes are 60..127, the Gaussian part stays far below
    assert abs(big.mean() - 0.01) < 0.004
    core = x[~big]
    assert abs(core.std() - 10.0) < 0.3
    clean = synth.gen_stream(synth.StreamSpec(L, 4096, 3.0, 0, 10.0, 0.0, 32, 32), 3, 0, 0).numpy()
    assert np.abs(clean).max() < 60


def test_emulator_bursts():
    L, on, period, phase = 1 << 20, 2048, 1 << 17, 5000
    m = synth.emulator_mask(L, on, period, phase).numpy()
    starts = np.flatnonzero(np.diff(m.astype(np.int8)) == 1) + 1
    assert starts[0] == phase and np.all(np.diff(starts) == period)
    assert m.sum() == on * len(starts) and not m[:phase].any()
    x = synth.gen_emulator_stream(L, 10.0, on, period, phase, 15.0, 0, 0).numpy().astype(np.float64)
    # 15 dB above the noise: burst samples have ~sqrt(1 + 10^1.5) times the spread (before saturation)
    ratio = x[m].std() / x[~m].std()
    assert 4.0 < ratio < 6.0
