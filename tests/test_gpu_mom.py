"""Median-of-MAD path (Eq. (3)) on the device against the oracle, bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import synth

pytestmark = pytest.mark.gpu
SENT = 0x5A


def _run(x_np, L, W, K, M, mom_k, seed, dev, inplace=False, stats=True):
    xd = torch.from_numpy(x_np.copy()).to(dev)
    yd = xd if inplace else torch.full_like(xd, SENT)
    y, st = rfi.mom_filter(xd, L, W, K, M, mom_k, seed=seed, y=yd, stats=stats)
    torch.cuda.synchronize()
    return y.cpu().numpy(), (rfi.stats_numpy(st) if st is not None else None)


def _check(x_np, L, W, K, M, mom_k, seed, y, st, padding=True):
    yo, sto = oracle.mom_filter_batch(x_np, L, W, K, M, mom_k, seed=seed)
    so, _, _, _ = rfi.layout(L, W)
    for s, (o, n) in enumerate(zip(so, L)):
        a, b = y[o:o + n], yo[o:o + n]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"stream {s} W={W[s]} mode={M[s]}: {len(bad)} differ, first {bad[0]}: "
                                 f"gpu {a[bad[0]]} oracle {b[bad[0]]}")
        if padding:
            pad = y[o + n:o + synth.align_up(n)].view(np.uint8)
            assert np.all(pad == SENT), f"padding of stream {s} written"
    if st is not None:
        if not np.array_equal(st, sto):
            bad = np.nonzero(st != sto)[0]
            raise AssertionError(f"stats differ at window {bad[0]}: {st[bad[0]]} vs {sto[bad[0]]}")


def _batch(specs, seed):
    x = synth.gen_packed(specs, seed, 31).numpy()
    return x, [s.length for s in specs], [s.window for s in specs], [s.k for s in specs], \
        [s.mode for s in specs]


# K around multiples of the 64-window count blocks: the search's partial
# blocks at both ends of a range take every length, on MAD sequences that
# start at arbitrary byte offsets (window counts 38, 150, 62, ...)
@pytest.mark.parametrize("mom_k", [1, 2, 7, 63, 64, 65, 129, 4096])
def test_mixed_batch(gpu, mom_k):
    specs = []
    for i, (W, L) in enumerate([(4096, 4096 * 37 + 100), (512, 512 * 150), (1000, 61_111),
                                (16384, 16384 * 5 + 3), (2048, 2048 * 70), (777, 50_000),
                                (8192, 8192 * 9), (1, 500), (13, 4_000), (1024, 1024 * 80 + 1)]):
        sig = 4.0 + 3.0 * i
        specs.append(synth.StreamSpec(L, W, [2.5, 3.0, 3.5][i % 3], i % 3, sig, 0.01, 8, 2000))
    x, L, W, K, M = _batch(specs, 40 + mom_k)
    y, st = _run(x, L, W, K, M, mom_k, 5, gpu)
    _check(x, L, W, K, M, mom_k, 5, y, st)


@pytest.mark.parametrize("k", [0.0, 0.5])
def test_noise_many_flagged(gpu, k):
    """Noise with most samples flagged (a threshold of at most one median of
    MADs): the replacement's pool of flagged dwords runs several rounds of its
    list in whole 16 KiB items (W 1024, 4096, 16384), and W 3000 draws sample
    by sample; equal to the oracle."""
    specs = [synth.StreamSpec(16384 * 3 + 500, W, k, rfi.NOISE, 12.0, 0.02, 8, 512)
             for W in (1024, 4096, 16384, 3000)]
    x, L, W, K, M = _batch(specs, 90 + int(k * 10))
    y, st = _run(x, L, W, K, M, 5, 7, gpu)
    _check(x, L, W, K, M, 5, 7, y, st)


def test_k1_equals_plain_filter(gpu):
    specs = [synth.StreamSpec(4096 * 40, 4096, 3.0, m, 10.0, 0.01, 8, 500) for m in (0, 1, 2)]
    x, L, W, K, M = _batch(specs, 3)
    y1, s1 = _run(x, L, W, K, M, 1, 9, gpu)
    xd = torch.from_numpy(x.copy()).to(gpu)
    y0, s0 = rfi.mad_filter(xd, L, W, K, M, seed=9, y=torch.full_like(xd, SENT))
    so = rfi.layout(L, W)[0]
    y0 = y0.cpu().numpy()
    for o, n in zip(so, L):
        assert np.array_equal(y1[o:o + n], y0[o:o + n])
    assert np.array_equal(s1, rfi.stats_numpy(s0))


def test_inplace_and_no_stats(gpu):
    specs = [synth.StreamSpec(100_000, 2048, 3.0, 2, 15.0, 0.02, 8, 3000),
             synth.StreamSpec(70_000, 700, 3.0, 0, 8.0, 0.01, 8, 900)]
    x, L, W, K, M = _batch(specs, 8)
    y, _ = _run(x, L, W, K, M, 16, 2, gpu, inplace=True, stats=False)
    _check(x, L, W, K, M, 16, 2, y, None, padding=False)


def test_long_bursts_caught(gpu):
    """A burst longer than half a window inflates that window's MAD so the
    plain filter misses it; the median of MADs keeps the threshold low."""
    W = 4096
    L = W * 64
    g = np.random.default_rng(1)
    x = np.clip(np.rint(g.normal(0, 8, L)), -128, 127)
    b0 = W * 40 + 100
    x[b0:b0 + 3000] = np.clip(x[b0:b0 + 3000] + g.choice([-80, 80], 3000), -128, 127)
    x = x.astype(np.int8)
    y_mad, st_mad = _run(x, [L], [W], [3.0], [0], 1, 0, gpu)
    y_mom, st_mom = _run(x, [L], [W], [3.0], [0], 32, 0, gpu)
    _check(x, [L], [W], [3.0], [0], 32, 0, y_mom, st_mom)
    assert st_mom[40]["n_flagged"] > 2500 > st_mad[40]["n_flagged"]


def test_full_size_sampled(gpu):
    """60 x 2^24, W 4096, K 4096 (the paper's median-of-MAD setting): two
    streams checked against the oracle, the rest by properties."""
    specs = synth.plain_scale(60, 1 << 24, 4096, rfi.CLIP)
    L = [s.length for s in specs]
    xd = synth.gen_packed(specs, 0, 77, device=gpu)
    y, st = rfi.mom_filter(xd, L, [4096] * 60, [3.0] * 60, [1] * 60, 4096, seed=3)
    torch.cuda.synchronize()
    so = rfi.layout(L, [4096] * 60)[0]
    stn = rfi.stats_numpy(st)
    for s in (0, 37):
        xs = xd[so[s]:so[s] + L[s]].cpu().numpy()
        # stream s sits behind s empty streams, so its key is s
        Ls = [0] * s + [L[s]]
        yo, sto = oracle.mom_filter_batch(xs, Ls, [4096] * (s + 1), 3.0, 1, 4096, seed=3)
        assert np.array_equal(y[so[s]:so[s] + L[s]].cpu().numpy(), yo[:L[s]])
        assert np.array_equal(stn[s * 4096:(s + 1) * 4096], sto)
    # CLIP never widens a sample's deviation beyond its window's threshold
    assert np.all(stn["threshold"] >= 0)


def test_arg_errors(gpu):
    xd = torch.zeros(4096, dtype=torch.int8, device=gpu)
    with pytest.raises(rfi.RfiError) as e:
        rfi.mom_filter(xd, [4096], [1024], [3.0], [1], 0)
    assert e.value.status == -1
    with pytest.raises(rfi.RfiError):
        rfi.mom_filter(xd, [4096], [0], [3.0], [1], 4)


def test_two_streams_same_signature(gpu):
    # the same argument signature on two HIP streams at once: each call has
    # its own temporaries, so both results equal the oracle's
    specs = [synth.StreamSpec(4096 * 300 + 77, 4096, 3.0, m, 8.0 + 3 * m, 0.01, 8, 3000) for m in (0, 1, 2)]
    xa, L, W, K, M = _batch(specs, 901)
    xb, _, _, _, _ = _batch(specs, 902)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    da, db = torch.from_numpy(xa).to(gpu), torch.from_numpy(xb).to(gpu)
    ya, yb = torch.empty_like(da), torch.empty_like(db)
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            _, sta = rfi.mom_filter(da, L, W, K, M, 64, seed=4, y=ya, stream=s1)
        with torch.cuda.stream(s2):
            _, stb = rfi.mom_filter(db, L, W, K, M, 64, seed=4, y=yb, stream=s2)
    torch.cuda.synchronize()
    _check(xa, L, W, K, M, 64, 4, ya.cpu().numpy(), rfi.stats_numpy(sta), padding=False)
    _check(xb, L, W, K, M, 64, 4, yb.cpu().numpy(), rfi.stats_numpy(stb), padding=False)


def _pack_np(parts):
    offs, total = synth.packed_offsets([len(p) for p in parts])
    out = np.zeros(max(total, 64), dtype=np.int8)
    for o, p in zip(offs, parts):
        out[o:o + len(p)] = p
    return out[:max(total, 1)], offs


@pytest.mark.parametrize("mom_k", [1, 7, 64, 65, 129, 300])
def test_carry_chained_equals_whole_stream(gpu, mom_k):
    # three streams cut at window boundaries into four calls each (the last
    # piece of each stream ends with a short window): the chained calls give
    # the bytes and statistics of one call over the whole streams
    Ws, Ks, Ms = [4096, 512, 1000], [3.0, 2.5, 3.5], [2, 1, 0]
    nwin = [[30, 1, 45, 20], [200, 7, 0, 90], [60, 60, 3, 40]]
    tails = [100, 17, 999]
    specs = [synth.StreamSpec(sum(nw) * W + t, W, k, m, 6.0 + 4 * i, 0.01, 8, 3000)
             for i, (nw, W, k, m, t) in enumerate(zip(nwin, Ws, Ks, Ms, tails))]
    xw, L, W, K, M = _batch(specs, 777 + mom_k)
    so = rfi.layout(L, W)[0]
    streams = [xw[so[s]:so[s] + L[s]] for s in range(3)]
    y_ref, st_ref = _run(xw, L, W, K, M, mom_k, 21, gpu)
    ns = 3
    hist = torch.zeros((ns, max(mom_k - 1, 1)), dtype=torch.uint8, device=gpu)
    hlen = torch.zeros(ns, dtype=torch.int32, device=gpu)
    pos = [0, 0, 0]
    outs = [[] for _ in range(ns)]
    stats = [[] for _ in range(ns)]
    for c in range(4):
        lens = [nwin[s][c] * W[s] + (tails[s] if c == 3 else 0) for s in range(ns)]
        parts = [streams[s][pos[s]:pos[s] + lens[s]] for s in range(ns)]
        xb, offs = _pack_np(parts)
        xd = torch.from_numpy(xb.copy()).to(gpu)
        absb = torch.tensor(pos, dtype=torch.int64, device=gpu)
        y, st = rfi.mom_filter_carry(xd, lens, W, K, M, mom_k, absb, hist if mom_k > 1 else None,
                                     hlen if mom_k > 1 else None, seed=21)
        torch.cuda.synchronize()
        yn = y.cpu().numpy()
        stn = rfi.stats_numpy(st) if st is not None else np.zeros(0, dtype=rfi.STATS_DTYPE)
        wo = rfi.layout(lens, W)[1]
        for s in range(ns):
            outs[s].append(yn[offs[s]:offs[s] + lens[s]])
            nws = (lens[s] + W[s] - 1) // W[s]
            stats[s].append(stn[wo[s]:wo[s] + nws])
            pos[s] += lens[s]
        if mom_k > 1:
            assert hlen.cpu().numpy().tolist() == [min(mom_k - 1, sum((nwin[s][j] + (1 if (j == 3 and tails[s]) else 0))
                                                                       for j in range(c + 1))) for s in range(ns)]
    wo_ref = rfi.layout(L, W)[1]
    for s in range(ns):
        got = np.concatenate(outs[s])
        assert np.array_equal(got, y_ref[so[s]:so[s] + L[s]]), (mom_k, s)
        nws = (L[s] + W[s] - 1) // W[s]
        assert np.array_equal(np.concatenate(stats[s]), st_ref[wo_ref[s]:wo_ref[s] + nws]), (mom_k, s)


def test_carry_errors(gpu):
    x = torch.zeros(4096, dtype=torch.int8, device=gpu)
    with pytest.raises(rfi.RfiError):
        rfi.mom_filter_carry(x, [4096], [512], [3.0], [0], 4, None, None, None)


def _oracle_stream(xs, s, W, k, m, mom_k, seed):
    # stream s alone, behind s empty streams, so that its noise key is s
    yo, sto = oracle.mom_filter_batch(xs, [0] * s + [len(xs)], [W] * (s + 1), [k] * (s + 1), [m] * (s + 1),
                                      mom_k, seed=seed)
    return yo[:len(xs)], sto


def test_large_mixed_batch_matches_oracle(gpu):
    # 72 M samples in six streams of mixed W, k and mode (noise in four):
    # every stream's bytes and statistics equal the oracle's
    Ws = [4096, 1000, 8192, 4096, 2048, 777]
    Ks = [3.0, 2.5, 3.5, 3.0, 4.0, 3.0]
    Ms = [2, 2, 0, 2, 1, 2]
    specs = [synth.StreamSpec(12_000_000 + 777 * i, Ws[i], Ks[i], Ms[i], 6.0 + 3 * i, 0.01, 8, 3000)
             for i in range(6)]
    L = [sp.length for sp in specs]
    xd = synth.gen_packed(specs, 5, 41, device=gpu)
    y, st = rfi.mom_filter(xd, L, Ws, Ks, Ms, 300, seed=9)
    torch.cuda.synchronize()
    so, wo, _, _ = rfi.layout(L, Ws)
    stn = rfi.stats_numpy(st)
    for s in range(6):
        xs = xd[so[s]:so[s] + L[s]].cpu().numpy()
        yo, sto = _oracle_stream(xs, s, Ws[s], Ks[s], Ms[s], 300, 9)
        assert np.array_equal(y[so[s]:so[s] + L[s]].cpu().numpy(), yo), s
        nw = (L[s] + Ws[s] - 1) // Ws[s]
        assert np.array_equal(stn[wo[s]:wo[s] + nw], sto), s


@pytest.mark.parametrize("mom_k", [1000, 4096])
def test_large_carry_equals_whole_stream(gpu, mom_k):
    # six noise streams in three calls of 3000 windows each (74 M samples
    # per call): bytes and statistics equal one call over the whole streams
    ns, W, nwc = 6, 4096, 3000
    specs = [synth.StreamSpec(3 * nwc * W, W, 3.0, 2, 7.0 + 2 * i, 0.01, 8, 3000) for i in range(ns)]
    L = [sp.length for sp in specs]
    xd = synth.gen_packed(specs, 6, 43, device=gpu)
    y_ref, st_ref = rfi.mom_filter(xd, L, [W] * ns, [3.0] * ns, [2] * ns, mom_k, seed=12)
    so = rfi.layout(L, [W] * ns)[0]
    hist = torch.zeros((ns, mom_k - 1), dtype=torch.uint8, device=gpu)
    hlen = torch.zeros(ns, dtype=torch.int32, device=gpu)
    n = nwc * W
    for c in range(3):
        xc = torch.cat([xd[so[s] + c * n:so[s] + (c + 1) * n] for s in range(ns)])
        absb = torch.full((ns,), c * n, dtype=torch.int64, device=gpu)
        yc, stc = rfi.mom_filter_carry(xc, [n] * ns, [W] * ns, [3.0] * ns, [2] * ns, mom_k, absb, hist, hlen,
                                       seed=12)
        for s in range(ns):
            assert torch.equal(yc[s * n:(s + 1) * n], y_ref[so[s] + c * n:so[s] + (c + 1) * n]), (c, s)
            assert torch.equal(stc[s * nwc:(s + 1) * nwc],
                               st_ref[s * 3 * nwc + c * nwc:s * 3 * nwc + (c + 1) * nwc]), (c, s)
    torch.cuda.synchronize()
    assert hlen.cpu().tolist() == [mom_k - 1] * ns


@pytest.mark.parametrize("carry", [False, True])
def test_large_batch_with_empty_streams(gpu, carry):
    # a 70 M-sample stream followed by empty ones: the batch is cut into
    # chunks of whole streams, three of which hold no window; the result
    # equals the oracle, with and without a carried history
    W, K = 4096, 300
    L = [70_000_000, 0, 0, 0]
    specs = [synth.StreamSpec(max(l, 1), W, 3.0, 2, 9.0, 0.01, 8, 3000) for l in L]
    xd = synth.gen_packed(specs[:1], 7, 45, device=gpu)
    n = len(L)
    if carry:
        hist = torch.zeros((n, K - 1), dtype=torch.uint8, device=gpu)
        hlen = torch.zeros(n, dtype=torch.int32, device=gpu)
        absb = torch.zeros(n, dtype=torch.int64, device=gpu)
        y, st = rfi.mom_filter_carry(xd, L, [W] * n, [3.0] * n, [2] * n, K, absb, hist, hlen, seed=4)
    else:
        y, st = rfi.mom_filter(xd, L, [W] * n, [3.0] * n, [2] * n, K, seed=4)
    torch.cuda.synchronize()
    xs = xd[:L[0]].cpu().numpy()
    yo, sto = _oracle_stream(xs, 0, W, 3.0, 2, K, 4)
    assert np.array_equal(y[:L[0]].cpu().numpy(), yo)
    assert np.array_equal(rfi.stats_numpy(st), sto)
    if carry:
        assert hlen.cpu().tolist() == [K - 1, 0, 0, 0]
