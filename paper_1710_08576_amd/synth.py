"""Seeded synthetic antenna streams: Gaussian noise plus impulsive RFI bursts.

This module only draws input data; it holds none of the filter's arithmetic,
so both the GPU path's tests and the CPU oracle's tests read its bytes.

The paper measures on GMRT antenna voltages and an analog RFI emulator,
neither of which is available; these streams stand in for them, shaped by the
RFI description of Sec. II-A (groups of strong impulses, 10-20 dB above the
system noise, superimposed on a Gaussian signal, making it heavy-tailed):

* int8 streams: ``x = sat(round(N(0, sigma^2)) + burst)``.  A burst covers a
  run of consecutive samples; it has one magnitude ``A ~ U{60..127}`` and a
  random sign per sample.  The number of bursts is ``round(frac * L / mean
  burst length)``, starts uniform over the stream, overlapping bursts add.
* int16 streams: Gaussian sigma 400 plus bursts on a fraction of samples whose
  values are ``50 * sigma * t`` with ``t`` Student-t (nu = 2), saturated.

Everything is drawn with ``torch`` generators so the same recipe runs on the
CPU (tests) or straight into device memory (GB-scale benchmarks).
"""
from __future__ import annotations

import dataclasses

import torch

I8_MIN, I8_MAX = -128, 127
I16_MIN, I16_MAX = -32768, 32767
ALIGN = 64  # stream starts are aligned to 64 elements in the packed layout


@dataclasses.dataclass
class StreamSpec:
    length: int
    window: int
    k: float
    mode: int
    sigma: float
    frac: float        # fraction of samples inside bursts
    burst_lo: int      # burst length range (inclusive)
    burst_hi: int
    dtype: str = "i8"  # "i8" or "i16"


def _gen(seed: int, tag: int, s: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((seed * 1_000_003 + tag * 10_007 + s * 101 + 17) & 0x7FFF_FFFF_FFFF_FFFF)
    return g


def _randint(g, lo, hi, size, device):
    return torch.randint(lo, hi + 1, size, generator=g, device=device)


def _burst_field(L, spec: StreamSpec, g, device):
    """Per-sample burst amplitude magnitude (0 outside bursts), int32."""
    mean_len = 0.5 * (spec.burst_lo + spec.burst_hi)
    nb = int(round(spec.frac * L / mean_len))
    field = torch.zeros(L + 1, dtype=torch.int32, device=device)
    if nb == 0 or L == 0:
        return field[:L]
    lens = _randint(g, spec.burst_lo, spec.burst_hi, (nb,), device)
    lens = torch.minimum(lens, torch.full_like(lens, L))
    starts = (torch.rand(nb, generator=g, device=device, dtype=torch.float64)
              * (L - lens + 1).to(torch.float64)).floor().to(torch.int64)
    amps = _randint(g, 60, 127, (nb,), device).to(torch.int32)
    field.index_add_(0, starts, amps)
    field.index_add_(0, starts + lens, -amps)
    return torch.cumsum(field, 0, dtype=torch.int32)[:L]


def gen_stream(spec: StreamSpec, seed: int, tag: int, s: int, device="cpu") -> torch.Tensor:
    """One stream of ``spec.length`` samples (int8 or int16 tensor)."""
    L = spec.length
    g = _gen(seed, tag, s, device)
    if spec.dtype == "i8":
        base = torch.randn(L, generator=g, device=device, dtype=torch.float32) * spec.sigma
        base = torch.round(base).to(torch.int32)
        amp = _burst_field(L, spec, g, device)
        sign = torch.randint(0, 2, (L,), generator=g, device=device, dtype=torch.int32) * 2 - 1
        v = base + amp * sign
        return torch.clamp(v, I8_MIN, I8_MAX).to(torch.int8)
    if spec.dtype == "i16":
        base = torch.randn(L, generator=g, device=device, dtype=torch.float32) * spec.sigma
        v = torch.round(base).to(torch.float64)
        mean_len = 0.5 * (spec.burst_lo + spec.burst_hi)
        nb = int(round(spec.frac * L / mean_len))
        if nb > 0 and L > 0:
            mask = torch.zeros(L + 1, dtype=torch.int32, device=device)
            lens = torch.minimum(_randint(g, spec.burst_lo, spec.burst_hi, (nb,), device),
                                 torch.full((nb,), L, device=device, dtype=torch.int64))
            starts = (torch.rand(nb, generator=g, device=device, dtype=torch.float64)
                      * (L - lens + 1).to(torch.float64)).floor().to(torch.int64)
            ones = torch.ones(nb, dtype=torch.int32, device=device)
            mask.index_add_(0, starts, ones)
            mask.index_add_(0, starts + lens, -ones)
            inside = torch.cumsum(mask, 0, dtype=torch.int32)[:L] > 0
            # Student-t, nu = 2: N(0,1) / sqrt(chi2_2 / 2), chi2_2 = -2 log U.
            z = torch.randn(L, generator=g, device=device, dtype=torch.float64)
            u = torch.rand(L, generator=g, device=device, dtype=torch.float64).clamp_min(1e-300)
            t = z / torch.sqrt(-torch.log(u))
            v = v + torch.where(inside, torch.round(50.0 * spec.sigma * t), torch.zeros_like(t))
        return torch.clamp(v, I16_MIN, I16_MAX).to(torch.int16)
    raise ValueError(spec.dtype)


def emulator_mask(length: int, on: int, period: int, phase: int = 0, device="cpu") -> torch.Tensor:
    """Boolean mask of the samples inside the periodic bursts of an RFI
    emulator: the first burst starts at sample ``phase``; sample i is inside
    iff i >= phase and (i - phase) mod period < on."""
    i = torch.arange(length, dtype=torch.int64, device=device)
    return (i >= phase) & (torch.remainder(i - phase, period) < on)


def gen_emulator_stream(length: int, sigma: float, on: int, period: int, phase: int,
                        burst_db: float, seed: int, s: int, device="cpu") -> torch.Tensor:
    """int8 stream with periodic broadband bursts, the synthetic stand-in for
    the analog RFI emulator of Sec. III-B (an on-period of 64 us every 2 s at
    800 Msample/s is on = 51 200 samples; the period is a parameter so that
    short streams still hold several bursts).  Outside a burst the samples
    are round(N(0, sigma^2)); inside, Gaussian noise whose power is
    ``burst_db`` above the system noise (the 10-20 dB of Sec. II-A) is added
    before rounding; the sum saturates to int8."""
    g = _gen(seed, 31, s, device)
    base = torch.randn(length, generator=g, device=device, dtype=torch.float32) * sigma
    extra = torch.randn(length, generator=g, device=device, dtype=torch.float32)
    extra = extra * (sigma * 10.0 ** (burst_db / 20.0))
    inside = emulator_mask(length, on, period, phase, device)
    v = torch.round(base + torch.where(inside, extra, torch.zeros_like(extra)))
    return torch.clamp(v, I8_MIN, I8_MAX).to(torch.int8)


def align_up(n: int, a: int = ALIGN) -> int:
    return (n + a - 1) // a * a


def packed_offsets(lengths):
    offs, total = [], 0
    for L in lengths:
        offs.append(total)
        total += align_up(int(L))
    return offs, total


def pack(streams, device="cpu") -> torch.Tensor:
    """Concatenate streams at 64-element-aligned offsets (zero padding)."""
    lengths = [int(t.numel()) for t in streams]
    offs, total = packed_offsets(lengths)
    dtype = streams[0].dtype if streams else torch.int8
    out = torch.zeros(max(total, ALIGN), dtype=dtype, device=device)
    for o, t in zip(offs, streams):
        out[o:o + t.numel()] = t.to(device)
    return out[:total] if total else out[:0]


def gen_packed(specs, seed: int, tag: int, device="cpu") -> torch.Tensor:
    """All streams of a config, drawn on ``device`` and packed there."""
    lengths = [s.length for s in specs]
    offs, total = packed_offsets(lengths)
    dt = torch.int8 if (not specs or specs[0].dtype == "i8") else torch.int16
    out = torch.zeros(max(total, ALIGN), dtype=dt, device=device)
    for s, (o, spec) in enumerate(zip(offs, specs)):
        out[o:o + spec.length] = gen_stream(spec, seed, tag, s, device)
    return out[:total]


# --------------------------------------------------------------------------
# The five workload configurations (sizes scale down for parity tests).
# --------------------------------------------------------------------------
ZERO, CLIP, NOISE = 0, 1, 2
WINDOW_CLASSES = (512, 1024, 2048, 4096, 8192, 16384)


def plain_one(length=1 << 20, window=4096, mode=CLIP):
    """1 stream, sigma 10, bursts on 0.1 % of samples, 32-sample bursts, k = 3."""
    return [StreamSpec(length, window, 3.0, mode, 10.0, 0.001, 32, 32)]


def plain_scale(n_streams=60, length=1 << 24, window=4096, mode=CLIP, seed=0):
    """60 streams (30 antennas x 2 pols); per stream sigma U[6,20], bursts on
    0.1-2 % of samples, lengths 8-512; k = 3; one mode for the whole batch."""
    g = torch.Generator().manual_seed(9001 + seed)
    out = []
    for _ in range(n_streams):
        sigma = 6.0 + 14.0 * float(torch.rand(1, generator=g))
        frac = 0.001 + 0.019 * float(torch.rand(1, generator=g))
        out.append(StreamSpec(length, window, 3.0, mode, sigma, frac, 8, 512))
    return out


def batching(n_streams=64, lo=1 << 18, hi=1 << 24, seed=0):
    """64 uneven streams: L U[2^18, 2^24], W from the six classes, k U[2.5,5],
    mixed modes; sigma and bursts as in the plain-scale workload."""
    g = torch.Generator().manual_seed(7001 + seed)
    out = []
    for _ in range(n_streams):
        L = int(torch.randint(lo, hi + 1, (1,), generator=g))
        W = WINDOW_CLASSES[int(torch.randint(0, 6, (1,), generator=g))]
        k = float(torch.tensor(2.5 + 2.5 * float(torch.rand(1, generator=g)),
                               dtype=torch.float32))
        mode = int(torch.randint(0, 3, (1,), generator=g))
        sigma = 6.0 + 14.0 * float(torch.rand(1, generator=g))
        frac = 0.001 + 0.019 * float(torch.rand(1, generator=g))
        out.append(StreamSpec(L, W, k, mode, sigma, frac, 8, 512))
    return out


def int16_path(n_streams=60, length=1 << 23, window=8192, mode=NOISE):
    """int16: sigma 400 plus Student-t (nu=2) bursts on 1 % of samples in
    32-sample bursts, scaled x50 (of sigma) and saturated; W = 8192, k = 3."""
    return [StreamSpec(length, window, 3.0, mode, 400.0, 0.01, 32, 32, "i16")
            for _ in range(n_streams)]


def serving_streams(n_streams=60, seed=0):
    """60 int8 streams for the serving loop; W in {1024..16384}, k = 3, CLIP."""
    g = torch.Generator().manual_seed(5001 + seed)
    out = []
    for _ in range(n_streams):
        W = (1024, 2048, 4096, 8192, 16384)[int(torch.randint(0, 5, (1,), generator=g))]
        sigma = 6.0 + 14.0 * float(torch.rand(1, generator=g))
        frac = 0.001 + 0.019 * float(torch.rand(1, generator=g))
        out.append(StreamSpec(0, W, 3.0, CLIP, sigma, frac, 8, 512))
    return out


def poisson_arrivals(n: int, mean_s: float, seed: int) -> list[float]:
    """Cumulative arrival times of a Poisson process with the given mean gap."""
    g = torch.Generator().manual_seed(3001 + seed)
    gaps = -torch.log(torch.rand(n, generator=g, dtype=torch.float64).clamp_min(1e-300)) * mean_s
    return torch.cumsum(gaps, 0).tolist()
