"""Device block power and improvement metric (Sec. III-A) against the
oracle, and the MAD / median-of-MAD breakdown on emulator bursts
(Sec. III-B) through the device path."""
import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

pytestmark = pytest.mark.gpu


def _packed(lengths, dtype, seed, extremes=True):
    total = sum(synth.align_up(L) for L in lengths)
    g = np.random.default_rng(seed)
    info = np.iinfo(dtype)
    x = g.integers(info.min, info.max + 1, max(total, 64)).astype(dtype)[:max(total, 64)]
    if extremes:
        off = 0
        for L in lengths:
            x[off:off + min(L, 3)] = info.min
            off += synth.align_up(L)
    return x


CASES = [
    # (lengths, block): tiny blocks on short streams, parts path on long ones
    ([0, 1, 63, 64, 65, 1000, 4097], 1),
    ([0, 1, 63, 64, 65, 1000, 4097], 7),
    ([5000, 0, 12345, 70000], 300),
    ([100_003, 65_536, 1, 200_000], 4096),
    ([300_000, 65_536, 65_537, 131_073], 65_536),
    ([300_000, 65_537, 5, 700_001], 65_537),
    ([(1 << 21) + 17, 3 << 20, 1 << 20], 1 << 20),
    ([5_000_000, 3], 3 * (1 << 20) + 5),
]


@pytest.mark.parametrize("dtype", [np.int8, np.int16])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_block_power_matches_oracle(gpu, dtype, case):
    lengths, block = CASES[case]
    x = _packed(lengths, dtype, 100 + case)
    xd = torch.from_numpy(x).to(gpu)
    got = rfi.block_power(xd, lengths, block).cpu().numpy()
    torch.cuda.synchronize()
    want = oracle.block_power(x, lengths, block)
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{len(bad)} blocks differ, first {bad[0]}: {got[bad[0]]} vs {want[bad[0]]}")


def test_block_power_saturated_int16_blocks(gpu):
    # every sample -32768: 2^30 per sample, 2^46 for a block of 2^16
    L = [1 << 20]
    x = np.full(1 << 20, -32768, dtype=np.int16)
    got = rfi.block_power(torch.from_numpy(x).to(gpu), L, 1 << 16).cpu().numpy()
    assert got.tolist() == [1 << 46] * 16


def test_block_power_errors(gpu):
    x = torch.zeros(1024, dtype=torch.int8, device=gpu)
    out = torch.zeros(16, dtype=torch.int64, device=gpu)
    for block in (0, -5, (1 << 30) + 1):
        with pytest.raises(rfi.RfiError):
            rfi.block_power(x, [1000], block, out=out)
    with pytest.raises(rfi.RfiError):  # power_out overlapping x
        rfi.block_power(x, [1000], 100, out=x.view(torch.int64)[:10])
    with pytest.raises(rfi.RfiError):  # unaligned x
        rfi.block_power(x[1:], [100], 10, out=out)
    # empty batch: nothing to do
    assert rfi.block_power(x, [0, 0], 10, out=out).numel() == 0


def _improvement_case(gpu, lengths, block, seg, seed):
    g = np.random.default_rng(seed)
    nb = rfi.n_blocks(lengths, block)
    pu = g.integers(1, 1 << 40, nb).astype(np.int64)
    pf = g.integers(1, 1 << 40, nb).astype(np.int64)
    got = rfi.improvement(torch.from_numpy(pu).to(gpu), torch.from_numpy(pf).to(gpu), lengths, block,
                          seg).cpu().numpy()
    want = oracle.improvement(pu, pf, lengths, block, seg)
    return got, want


@pytest.mark.parametrize("seg", [1, 2, 16, 300])
def test_improvement_matches_oracle(gpu, seg):
    lengths = [1000 * 64, 0, 64 * 17 + 5, 64 * 5000, 64 * 2]
    got, want = _improvement_case(gpu, lengths, 64, seg, seg)
    # same definition, summation order differs (tree over segments)
    fin = np.isfinite(want)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    np.testing.assert_allclose(got[fin], want[fin], rtol=1e-12, atol=1e-12)
    assert np.array_equal(got[~fin & ~np.isnan(want)], want[~fin & ~np.isnan(want)])


def test_improvement_closed_forms(gpu):
    pu = torch.tensor([10, 30] * 8, dtype=torch.int64, device=gpu)
    pf = torch.tensor([18, 22] * 8, dtype=torch.int64, device=gpu)
    # hand-worked: S_U = 20 / 40, S_F = 4 / 40, 10 log10(S_U / S_F) = 10 log10 5
    r = rfi.improvement(pu, pf, [80], 5, 16).cpu().numpy()[0]
    assert r[0] == pytest.approx(0.5, rel=1e-15) and r[1] == pytest.approx(0.1, rel=1e-15)
    assert r[2] == pytest.approx(6.989700043360188, abs=1e-12)
    r = rfi.improvement(pf, pu, [80], 5, 16).cpu().numpy()[0]
    assert r[2] == pytest.approx(-6.989700043360188, abs=1e-12)
    r = rfi.improvement(pu, pu, [80], 5, 16).cpu().numpy()[0]
    assert r[2] == 0.0
    # a filtered power with no deviation: S_F = 0, improvement +inf
    const = torch.full((16,), 7, dtype=torch.int64, device=gpu)
    r = rfi.improvement(pu, const, [80], 5, 16).cpu().numpy()[0]
    assert r[1] == 0.0 and r[2] == np.inf


def test_improvement_ranking_plain_scale_full_size(gpu):
    # The plain-scale batch (60 x 2^24 int8, W 4096, k 3), integrated over
    # blocks of 2^20 samples (1.31 ms at 800 Msample/s), segments of 16:
    # zero and noise replacement improve far more than clipping (Sec. III-B).
    ns, L, block, seg = 60, 1 << 24, 1 << 20, 16
    specs = synth.plain_scale(ns, L, 4096, synth.ZERO)
    lengths = [s.length for s in specs]
    x = synth.gen_packed(specs, 0, 100, device=gpu)
    pu = rfi.block_power(x, lengths, block)
    so, _, _, _ = rfi.layout(lengths, [4096] * ns)
    res = {}
    for name, m in (("zero", 0), ("clip", 1), ("noise", 2)):
        y, _ = rfi.mad_filter(x, lengths, [4096] * ns, [3.0] * ns, [m] * ns, seed=1, stats=False)
        pf = rfi.block_power(y, lengths, block)
        res[name] = rfi.improvement(pu, pf, lengths, block, seg).cpu().numpy()
        # sampled streams: block powers and metric against the oracle
        for s in (0, 37, 59):
            xs = x[so[s]:so[s] + L].cpu().numpy()
            ys = y[so[s]:so[s] + L].cpu().numpy()
            pu_o, pf_o = oracle.block_power(xs, [L], block), oracle.block_power(ys, [L], block)
            assert np.array_equal(pu[s * 16:(s + 1) * 16].cpu().numpy(), pu_o)
            assert np.array_equal(pf[s * 16:(s + 1) * 16].cpu().numpy(), pf_o)
            want = oracle.improvement(pu_o, pf_o, [L], block, seg)[0]
            np.testing.assert_allclose(res[name][s], want, rtol=1e-12, atol=1e-12)
    del x
    imp = {k: v[:, 2] for k, v in res.items()}
    assert np.all(imp["clip"] > 0.5)
    assert np.all(imp["zero"] > imp["clip"] + 2.0)
    assert np.all(imp["noise"] > imp["clip"] + 2.0)
    assert abs(float(np.median(imp["zero"] - imp["noise"]))) < 3.0


@pytest.mark.parametrize("on", [2048, 8192, 51200])
def test_breakdown_on_emulator_bursts_matches_oracle(gpu, on):
    # Two emulator streams (first burst after the 256-window history of the
    # median of MAD has filled): the device's MAD (W 16384) and median-of-MAD
    # (W 4096, 256 windows) outputs equal the oracle's, so their detection
    # fractions on the burst samples do too; MAD loses the long bursts.
    L, period, phase = 1 << 22, 1 << 20, 256 * 4096 + 1000
    xs = [synth.gen_emulator_stream(L, 10.0 + 4 * s, on, period, phase, 15.0, 0, s).numpy() for s in range(2)]
    x = np.concatenate(xs)
    mask = np.concatenate([synth.emulator_mask(L, on, period, phase).numpy()] * 2)
    xd = torch.from_numpy(x).to(gpu)
    y_mad, _ = rfi.mad_filter(xd, [L, L], [16384] * 2, [3.0] * 2, [rfi.CLIP] * 2, seed=3, stats=False)
    y_mom, _ = rfi.mom_filter(xd, [L, L], [4096] * 2, [3.0] * 2, [rfi.CLIP] * 2, 256, seed=3, stats=False)
    y_mad, y_mom = y_mad.cpu().numpy(), y_mom.cpu().numpy()
    yo_mad, _ = oracle.filter_batch(x, [L, L], [16384] * 2, 3.0, oracle.CLIP, seed=3)
    yo_mom, _ = oracle.mom_filter_batch(x, [L, L], [4096] * 2, 3.0, oracle.CLIP, 256, seed=3)
    assert np.array_equal(y_mad, yo_mad)
    assert np.array_equal(y_mom, yo_mom)
    det_mad = float((y_mad != x)[mask].mean())
    det_mom = float((y_mom != x)[mask].mean())
    if on <= 2048:
        assert det_mad > 0.9 * det_mom
    elif on >= 51200:
        assert det_mad < 0.15 * det_mom


def test_block_power_two_streams_same_signature(gpu):
    # blocks of 3 * 2^20 go through the parts buffer, which is per stream
    lengths, block = [5_000_000, 3_000_001], 3 << 20
    xa = _packed(lengths, np.int8, 501)
    xb = _packed(lengths, np.int8, 502)
    da, db = torch.from_numpy(xa).to(gpu), torch.from_numpy(xb).to(gpu)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    nb = rfi.n_blocks(lengths, block)
    pa = torch.empty(nb, dtype=torch.int64, device=gpu)
    pb = torch.empty(nb, dtype=torch.int64, device=gpu)
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            rfi.block_power(da, lengths, block, out=pa, stream=s1)
        with torch.cuda.stream(s2):
            rfi.block_power(db, lengths, block, out=pb, stream=s2)
    torch.cuda.synchronize()
    assert np.array_equal(pa.cpu().numpy(), oracle.block_power(xa, lengths, block))
    assert np.array_equal(pb.cpu().numpy(), oracle.block_power(xb, lengths, block))
