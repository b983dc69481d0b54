"""Serving runtime: blocks of many streams, device carry, admission, replay.

The contract under test: the concatenated output of a stream served block by
block (with any block sizes, interleaved with other streams, through any
number of lanes and batches, across a snapshot/restore, ending with a flush)
equals the oracle's output for the whole stream as one batch -- the same
windows, the same statistics, the same noise draws -- and a stream's result
is the same alone and in the mix.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1710_08576_amd as rfi
from paper_1710_08576_amd import _lib, synth

SEED = 77


def make_streams(specs, seed, tag=5):
    xs = [synth.gen_stream(s, seed, tag, i).numpy() for i, s in enumerate(specs)]
    return xs


def oracle_streams(xs, specs, seed):
    """Per-stream oracle outputs and stats (stream index = stream id)."""
    L = [len(x) for x in xs]
    W = [s.window for s in specs]
    so, wo, total, n = rfi.layout(L, W)
    dt = xs[0].dtype
    packed = np.zeros(n, dtype=dt)
    for o, x in zip(so, xs):
        packed[o:o + len(x)] = x
    y, st = oracle.filter_batch(packed, L, W, [s.k for s in specs], [s.mode for s in specs],
                                seed=seed)
    ys, sts = [], []
    for i, x in enumerate(xs):
        ys.append(y[so[i]:so[i] + len(x)])
        nw = (len(x) + W[i] - 1) // W[i]
        sts.append(st[wo[i]:wo[i] + nw])
    return ys, sts


def split_sizes(total, rng, choices):
    sizes = []
    left = total
    while left > 0:
        n = min(left, int(rng.choice(choices)))
        sizes.append(n)
        left -= n
    return sizes


class Served:
    """Drives a server block by block and collects each stream's output."""

    def __init__(self, srv, dev, specs, dtype):
        self.srv, self.dev, self.specs, self.dtype = srv, dev, specs, dtype
        self.keep = []  # (sid, ticket, out, stats) in submit order
        self.outs = {i: [] for i in range(len(specs))}
        self.stats = {i: [] for i in range(len(specs))}

    def submit(self, sid, block_np, with_stats=True):
        n = len(block_np)
        W = self.specs[sid].window
        blk = torch.from_numpy(block_np.copy()).to(self.dev) if n else \
            torch.empty(0, dtype=self.dtype, device=self.dev)
        fill = 0x5A if self.dtype == torch.int8 else 0x5A5A
        out = torch.full((n + W - 1,), fill, dtype=self.dtype, device=self.dev)
        st = torch.full((self.srv.stats_entries(sid, n), 4), -7, dtype=torch.int32,
                        device=self.dev) if with_stats else None
        while True:
            t = self.srv.try_submit(sid, blk, out, st, n=n)
            if t is not None:
                break
            self.srv.sync()
        self.keep.append((sid, t, blk, out, st))
        return t

    def collect(self):
        self.srv.sync()
        for sid, t, _, out, st in self.keep:
            done, se, we = self.srv.poll(t)
            assert done
            o = out.cpu().numpy()
            self.outs[sid].append(o[:se])
            pad = o[se:].view(np.uint8 if o.dtype == np.int8 else np.uint16)
            assert np.all(pad == (0x5A if o.dtype == np.int8 else 0x5A5A)), "wrote past emitted"
            if st is not None:
                self.stats[sid].append(rfi.stats_numpy(st[:we]))
        self.keep = []

    def flush(self, sid):
        W = self.specs[sid].window
        out = torch.zeros(W, dtype=self.dtype, device=self.dev)
        st = torch.full((1, 4), -7, dtype=torch.int32, device=self.dev)
        n = self.srv.flush(sid, out, st)
        if n:
            self.outs[sid].append(out[:n].cpu().numpy())
            self.stats[sid].append(rfi.stats_numpy(st))
        return n

    def result(self, sid):
        npdt = np.int8 if self.dtype == torch.int8 else np.int16
        y = np.concatenate(self.outs[sid]) if self.outs[sid] else np.zeros(0, npdt)
        st = np.concatenate(self.stats[sid]) if self.stats[sid] else np.zeros(0, rfi.STATS_DTYPE)
        return y, st


def assert_same(y, st, yo, sto, what):
    assert len(y) == len(yo), f"{what}: {len(y)} samples emitted, expected {len(yo)}"
    if not np.array_equal(y, yo):
        bad = np.nonzero(y != yo)[0]
        raise AssertionError(f"{what}: {len(bad)} samples differ, first at {bad[0]}: "
                             f"served {y[bad[0]]} oracle {yo[bad[0]]}")
    if st is not None:
        assert len(st) == len(sto), f"{what}: {len(st)} windows, expected {len(sto)}"
        if not np.array_equal(st, sto):
            bad = np.nonzero(st != sto)[0]
            raise AssertionError(f"{what}: stats differ at window {bad[0]}: "
                                 f"{st[bad[0]]} vs {sto[bad[0]]}")


def mixed_specs(dtype="i8"):
    sig = 10.0 if dtype == "i8" else 400.0
    out = []
    for W, mode, k in [(4096, 2, 3.0), (1000, 1, 2.5), (512, 0, 3.5), (16384, 2, 3.0),
                       (4096, 1, 3.0), (777, 2, 4.0), (2048, 0, 3.0), (8192, 2, 3.0)]:
        out.append(synth.StreamSpec(0, W, k, mode, sig, 0.01, 8, 200, dtype))
    return out


def run_mix(dev, specs, xs, seed, sizes_per_stream, n_lanes=2, schedule="fused", max_batch=64,
            order_rng=None, dtype=torch.int8):
    srv = rfi.Server(elem_size=1 if dtype == torch.int8 else 2, max_streams=len(specs),
                     max_inflight=64, max_batch=max_batch, hbm_budget_bytes=1 << 32, seed=seed,
                     n_lanes=n_lanes, schedule=schedule)
    for i, s in enumerate(specs):
        srv.add_stream(i, s.window, s.k, s.mode)
    drv = Served(srv, dev, specs, dtype)
    queues = []
    for i, sizes in sizes_per_stream.items():
        pos = 0
        q = []
        for n in sizes:
            q.append((i, xs[i][pos:pos + n]))
            pos += n
        queues.append(q)
    # interleave the streams' blocks (each stream keeps its own order)
    rng = order_rng or np.random.default_rng(0)
    while any(queues):
        live = [q for q in queues if q]
        q = live[int(rng.integers(len(live)))]
        sid, blk = q.pop(0)
        drv.submit(sid, blk)
        if rng.random() < 0.2:
            srv.dispatch()
    drv.collect()
    for i in sizes_per_stream:
        drv.flush(i)
    res = {i: drv.result(i) for i in sizes_per_stream}
    counters = srv.counters()
    srv.close()
    return res, counters


# --------------------------------------------------------------------------
# host-only checks (no device calls)
# --------------------------------------------------------------------------

def test_server_config_rejected_on_host():
    lib = _lib.load()
    h = ctypes.c_void_p()
    bad = [
        _lib.ServerConfig(3, 4, 8, 8, 1 << 30, 0, 1, 3),     # elem size
        _lib.ServerConfig(1, 0, 8, 8, 1 << 30, 0, 1, 3),     # no streams
        _lib.ServerConfig(1, 4, 0, 8, 1 << 30, 0, 1, 3),     # no in-flight slots
        _lib.ServerConfig(1, 4, 8, 0, 1 << 30, 0, 1, 3),     # empty batches
        _lib.ServerConfig(1, 4, 8, 8, 1 << 30, 0, 0, 3),     # no lanes
        _lib.ServerConfig(1, 4, 8, 8, 1 << 30, 0, 1, 1),     # split schedule not served
    ]
    for cfg in bad:
        assert lib.rfi_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
        assert not h.value
    assert lib.rfi_server_create(None, ctypes.byref(h)) == -1
    assert lib.rfi_server_destroy(None) == 0
    assert lib.rfi_server_submit(None, 0, None, None, 0, None, None) == -1
    assert lib.rfi_server_replay(None, 0, None, None, None, None, None, None, None, None) == -1


# --------------------------------------------------------------------------
# device parity
# --------------------------------------------------------------------------

@pytest.mark.gpu
@pytest.mark.parametrize("n_lanes,schedule", [(1, "fused"), (3, "fused"), (2, "fused_persist")])
def test_split_invariance_int8(gpu, n_lanes, schedule):
    specs = mixed_specs()
    rng = np.random.default_rng(11)
    lengths = [int(rng.integers(40_000, 120_000)) for _ in specs]
    for s, L in zip(specs, lengths):
        s.length = L
    xs = make_streams(specs, SEED)
    yo, sto = oracle_streams(xs, specs, SEED)
    # block sizes: empty, tiny, sub-window, several windows, whole tiles, odd
    choices = [0, 1, 17, 300, 1000, 4096, 8192, 16384, 16384 * 2, 5000, 12345]
    sizes = {i: split_sizes(len(x), rng, choices) for i, x in enumerate(xs)}
    res, cnt = run_mix(gpu, specs, xs, SEED, sizes, n_lanes=n_lanes, schedule=schedule,
                       order_rng=np.random.default_rng(3))
    for i in range(len(specs)):
        assert_same(*res[i], yo[i], sto[i], f"stream {i} W={specs[i].window} mode={specs[i].mode}")
    assert cnt["admitted"] == cnt["completed"] == sum(len(v) for v in sizes.values())


@pytest.mark.gpu
def test_tile_path_with_carry_int8(gpu):
    """Blocks that keep the carry a multiple of 16 samples, so bodies after a
    head window take the tile path at 16-byte-aligned offsets."""
    specs = [synth.StreamSpec(0, W, 3.0, m, 12.0, 0.02, 8, 300)
             for W, m in [(4096, 2), (4096, 0), (512, 2), (16384, 1), (2048, 2), (8192, 2)]]
    rng = np.random.default_rng(5)
    for s in specs:
        s.length = 16384 * 12 + 48
    xs = make_streams(specs, SEED + 1)
    yo, sto = oracle_streams(xs, specs, SEED + 1)
    choices = [16384 + 16, 16384 * 2 - 32, 4096 + 48, 16384 * 3, 64]
    sizes = {i: split_sizes(len(x), rng, choices) for i, x in enumerate(xs)}
    res, _ = run_mix(gpu, specs, xs, SEED + 1, sizes, n_lanes=2)
    for i in range(len(specs)):
        assert_same(*res[i], yo[i], sto[i], f"stream {i} W={specs[i].window}")


@pytest.mark.gpu
def test_split_invariance_int16(gpu):
    specs = mixed_specs("i16")
    rng = np.random.default_rng(21)
    for s in specs:
        s.length = int(rng.integers(30_000, 80_000))
    xs = make_streams(specs, SEED + 2)
    yo, sto = oracle_streams(xs, specs, SEED + 2)
    choices = [0, 3, 700, 8192, 8192 * 3, 9000, 20000]
    sizes = {i: split_sizes(len(x), rng, choices) for i, x in enumerate(xs)}
    res, _ = run_mix(gpu, specs, xs, SEED + 2, sizes, n_lanes=2, dtype=torch.int16)
    for i in range(len(specs)):
        assert_same(*res[i], yo[i], sto[i], f"int16 stream {i} W={specs[i].window}")


@pytest.mark.gpu
def test_alone_equals_in_mix(gpu):
    """Stream 5's result is the same served alone and among seven others."""
    specs = mixed_specs()
    rng = np.random.default_rng(31)
    for s in specs:
        s.length = 60_000
    xs = make_streams(specs, SEED)
    choices = [1000, 4096, 16384, 333, 20000]
    sizes = {i: split_sizes(len(x), rng, choices) for i, x in enumerate(xs)}
    mix, _ = run_mix(gpu, specs, xs, SEED, sizes, n_lanes=2)
    alone, _ = run_mix(gpu, specs, xs, SEED, {5: sizes[5]}, n_lanes=2)
    # and with other block sizes for stream 5 itself
    alone2, _ = run_mix(gpu, specs, xs, SEED, {5: split_sizes(60_000, rng, [7, 60_000])},
                        n_lanes=1)
    for other in (alone, alone2):
        assert np.array_equal(mix[5][0], other[5][0])
        assert np.array_equal(mix[5][1], other[5][1])
    yo, sto = oracle_streams(xs, specs, SEED)
    assert_same(*mix[5], yo[5], sto[5], "stream 5")


@pytest.mark.gpu
def test_snapshot_restore(gpu):
    specs = mixed_specs()[:4]
    for s in specs:
        s.length = 50_000
    xs = make_streams(specs, SEED + 3)
    yo, sto = oracle_streams(xs, specs, SEED + 3)
    cut = 23_456

    def new_server():
        srv = rfi.Server(elem_size=1, max_streams=4, seed=SEED + 3, n_lanes=2)
        for i, s in enumerate(specs):
            srv.add_stream(i, s.window, s.k, s.mode)
        return srv

    srv = new_server()
    drv = Served(srv, gpu, specs, torch.int8)
    for i in range(4):
        for a in range(0, cut, 5000):
            drv.submit(i, xs[i][a:min(a + 5000, cut)])
    drv.collect()
    snaps = {i: srv.snapshot(i) for i in range(4)}
    first = {i: drv.result(i) for i in range(4)}
    srv.close()
    for i in range(4):
        W = specs[i].window
        assert snaps[i][0] == cut // W * W
        assert np.array_equal(snaps[i][1], xs[i][cut // W * W:cut])

    srv = new_server()
    for i in range(4):
        srv.restore(i, *snaps[i])
    drv = Served(srv, gpu, specs, torch.int8)
    for i in range(4):
        drv.submit(i, xs[i][cut:])
    drv.collect()
    for i in range(4):
        drv.flush(i)
        y2, st2 = drv.result(i)
        y = np.concatenate([first[i][0], y2])
        st = np.concatenate([first[i][1], st2])
        assert_same(y, st, yo[i], sto[i], f"restored stream {i}")
    srv.close()


@pytest.mark.gpu
def test_restore_unaligned_index(gpu):
    """A restored stream whose next index is not a multiple of 16: windows
    follow the oracle at that absolute index (tile path must not be used)."""
    W, start = 4096, 1_000_003
    spec = synth.StreamSpec(W * 6, W, 3.0, synth.NOISE, 15.0, 0.02, 8, 300)
    x = synth.gen_stream(spec, SEED, 9, 0).numpy()
    srv = rfi.Server(elem_size=1, max_streams=1, seed=SEED, n_lanes=1)
    srv.add_stream(0, W, 3.0, synth.NOISE)
    srv.restore(0, start, np.zeros(0, np.int8))
    drv = Served(srv, gpu, [spec], torch.int8)
    drv.submit(0, x)
    drv.collect()
    y, st = drv.result(0)
    for w in range(6):
        yo, so = oracle.window(x[w * W:(w + 1) * W], 3.0, synth.NOISE, abs_start=start + w * W,
                               stream=0, seed=SEED)
        assert np.array_equal(y[w * W:(w + 1) * W], yo), f"window {w}"
        assert st[w] == so
    srv.close()


@pytest.mark.gpu
def test_admission_budget_and_inflight(gpu):
    W = 4096
    n = 1 << 16
    x = torch.zeros(n, dtype=torch.int8, device=gpu)
    outs = [torch.empty(n + W - 1, dtype=torch.int8, device=gpu) for _ in range(4)]
    # one block: n in + (n + W - 1) out + ceil((n + W - 1) / W) stats
    one = n + n + W - 1 + ((n + 2 * W - 2) // W) * 16
    srv = rfi.Server(elem_size=1, max_streams=2, max_inflight=8, hbm_budget_bytes=one + 10,
                     n_lanes=1)
    srv.add_stream(0, W, 3.0, 1)
    srv.add_stream(1, W, 3.0, 1)
    t0 = srv.submit(0, x, outs[0])
    # submit never retires work: the second block exceeds the budget
    assert srv.try_submit(1, x, outs[1]) is None
    srv.sync()
    assert srv.poll(t0)[0]
    t1 = srv.submit(1, x, outs[1])
    srv.sync()
    c = srv.counters()
    assert c["admitted"] == 2 and c["refused"] == 1 and c["completed"] == 2
    srv.close()
    # in-flight limit
    srv = rfi.Server(elem_size=1, max_streams=2, max_inflight=2, hbm_budget_bytes=1 << 30,
                     n_lanes=1)
    srv.add_stream(0, W, 3.0, 1)
    ts = [srv.submit(0, x, outs[i]) for i in range(2)]
    assert srv.try_submit(0, x, outs[2]) is None
    srv.sync()
    ts.append(srv.submit(0, x, outs[2]))
    srv.sync()
    assert all(srv.poll(t)[0] for t in ts)
    s0, d0 = srv.ticket_times(ts[0])
    assert 0 < s0 <= d0
    assert t1 > t0
    srv.close()


@pytest.mark.gpu
def test_submit_errors(gpu):
    W = 1024
    srv = rfi.Server(elem_size=1, max_streams=2, n_lanes=1)
    srv.add_stream(0, W, 3.0, 1)
    x = torch.zeros(4096, dtype=torch.int8, device=gpu)
    out = torch.empty(4096 + W, dtype=torch.int8, device=gpu)
    with pytest.raises(rfi.RfiError) as e:
        srv.submit(1, x, out)          # not registered
    assert e.value.status == -1
    with pytest.raises(rfi.RfiError) as e:
        srv.submit(0, x[1:], out, n=100)  # misaligned block
    assert e.value.status == -2
    with pytest.raises(rfi.RfiError):
        srv.add_stream(0, W, 3.0, 1)   # twice
    with pytest.raises(rfi.RfiError):
        srv.add_stream(1, 0, 3.0, 1)   # bad window
    with pytest.raises(rfi.RfiError):
        srv.restore(0, 0, np.zeros(W, np.int8))  # carry must be < W
    srv.close()


@pytest.mark.gpu
def test_replay_poisson(gpu):
    """Real-time replay of Poisson arrivals: outputs equal the oracle and
    every block gets a latency."""
    specs = [synth.StreamSpec(0, W, 3.0, m, 10.0, 0.01, 8, 300)
             for W, m in [(1024, 1), (4096, 2), (16384, 1), (2048, 0), (3000, 2), (8192, 1)]]
    nblk, bl = 12, 1 << 15
    for s in specs:
        s.length = nblk * bl + 1234
    xs = make_streams(specs, SEED + 4)
    yo, sto = oracle_streams(xs, specs, SEED + 4)
    srv = rfi.Server(elem_size=1, max_streams=len(specs), max_inflight=16,
                     hbm_budget_bytes=1 << 24, seed=SEED + 4, n_lanes=2)
    for i, s in enumerate(specs):
        srv.add_stream(i, s.window, s.k, s.mode)
    ev = []
    for i, s in enumerate(specs):
        t = np.cumsum(np.random.default_rng(100 + i).exponential(40e3, nblk + 1))
        pos = 0
        for b in range(nblk + 1):
            n = bl if b < nblk else len(xs[i]) - pos
            ev.append((int(t[b]), i, pos, n))
            pos += n
    ev.sort()
    blocks = [torch.from_numpy(xs[i][p:p + n].copy()).to(gpu) for _, i, p, n in ev]
    outs = [torch.full((n + specs[i].window - 1,), 0x5A, dtype=torch.int8, device=gpu)
            for _, i, p, n in ev]
    stats = [torch.full(((n + 2 * specs[i].window - 2) // specs[i].window, 4), -7,
                        dtype=torch.int32, device=gpu) for _, i, p, n in ev]
    lat, em = srv.replay([e[1] for e in ev], [e[0] for e in ev], blocks, outs, stats)
    assert np.all(lat > 0)
    ys = {i: [] for i in range(len(specs))}
    sts = {i: [] for i in range(len(specs))}
    for (_, i, _, _), o, st, e in zip(ev, outs, stats, em):
        W = specs[i].window
        ys[i].append(o[:e].cpu().numpy())
        sts[i].append(rfi.stats_numpy(st[:e // W]))
    drv = Served(srv, gpu, specs, torch.int8)
    for i in range(len(specs)):
        drv.flush(i)
        fy, fs = drv.result(i)
        y = np.concatenate(ys[i] + [fy])
        st = np.concatenate(sts[i] + [fs])
        assert_same(y, st, yo[i], sto[i], f"replayed stream {i}")
    c = srv.counters()
    assert c["completed"] == len(ev)
    srv.close()


@pytest.mark.gpu
@pytest.mark.parametrize("max_batch", [5, 64])
def test_burst_batches_chain_carries(gpu, max_batch):
    """Every block ready at once: the first batches hold several blocks of
    one stream, whose head windows read the previous block's tail in the
    same launch, including blocks shorter than a window."""
    specs = mixed_specs()
    rng = np.random.default_rng(41)
    for s in specs:
        s.length = 70_000
    xs = make_streams(specs, SEED + 5)
    yo, sto = oracle_streams(xs, specs, SEED + 5)
    srv = rfi.Server(elem_size=1, max_streams=len(specs), max_inflight=4096, max_batch=max_batch,
                     hbm_budget_bytes=1 << 32, seed=SEED + 5, n_lanes=2)
    for i, s in enumerate(specs):
        srv.add_stream(i, s.window, s.k, s.mode)
    ev = []
    for i in range(len(specs)):
        pos = 0
        for n in split_sizes(70_000, rng, [100, 2000, 4096, 9000, 16384, 33]):
            ev.append((i, pos, n))
            pos += n
    blocks = [torch.from_numpy(xs[i][p:p + n].copy()).to(gpu) for i, p, n in ev]
    outs = [torch.full((n + specs[i].window - 1,), 0x5A, dtype=torch.int8, device=gpu)
            for i, p, n in ev]
    stats = [torch.full(((n + 2 * specs[i].window - 2) // specs[i].window, 4), -7,
                        dtype=torch.int32, device=gpu) for i, p, n in ev]
    lat, em = srv.replay([e[0] for e in ev], [0] * len(ev), blocks, outs, stats)
    c = srv.counters()
    assert c["launches"] < len(ev)  # several blocks per batch
    ys = {i: [] for i in range(len(specs))}
    sts = {i: [] for i in range(len(specs))}
    for (i, _, _), o, st, e in zip(ev, outs, stats, em):
        ys[i].append(o[:e].cpu().numpy())
        sts[i].append(rfi.stats_numpy(st[:e // specs[i].window]))
    drv = Served(srv, gpu, specs, torch.int8)
    for i in range(len(specs)):
        drv.flush(i)
        fy, fs = drv.result(i)
        assert_same(np.concatenate(ys[i] + [fy]), np.concatenate(sts[i] + [fs]), yo[i], sto[i],
                    f"burst stream {i} W={specs[i].window}")
    srv.close()


def _served_streams(specs, xs, ev_blocks, outs_host, stride, em):
    """Per-stream concatenated outputs of blocks replayed into one output
    buffer per stream at a fixed stride (ev_blocks: (stream, slot) in
    arrival order)."""
    ys = {i: [] for i in range(len(specs))}
    for (i, slot), e in zip(ev_blocks, em):
        ys[i].append(outs_host[i][slot * stride:slot * stride + e])
    return ys


@pytest.mark.gpu
def test_ticket_records_bounded_over_1e5_replayed_blocks(gpu):
    """10^5 blocks replayed (every block ready at once, so admission runs at
    its limit throughout): the ticket records retire as blocks complete, so
    the live count never exceeds the in-flight limit and ends at zero, and
    every stream's output equals the oracle's."""
    specs = [synth.StreamSpec(0, W, 3.0, m, 10.0, 0.01, 8, 200)
             for W, m in [(1024, 1), (4096, 2), (2048, 0), (3000, 2)]]
    nblk, n = 25_000, 2048
    for s in specs:
        s.length = nblk * n
    xs = make_streams(specs, SEED + 6)
    yo, _ = oracle_streams(xs, specs, SEED + 6)
    max_inflight = 64
    srv = rfi.Server(elem_size=1, max_streams=len(specs), max_inflight=max_inflight, max_batch=16,
                     hbm_budget_bytes=1 << 32, seed=SEED + 6, n_lanes=2)
    for i, s in enumerate(specs):
        srv.add_stream(i, s.window, s.k, s.mode)
    xd = [torch.from_numpy(x).to(gpu) for x in xs]
    stride = (n + 4096 - 1 + 15) // 16 * 16
    outs = [torch.full((nblk * stride,), 0x5A, dtype=torch.int8, device=gpu) for _ in specs]
    sid = np.tile(np.arange(len(specs), dtype=np.uint32), nblk)
    slot = np.repeat(np.arange(nblk, dtype=np.int64), len(specs))
    bp = np.array([xd[i].data_ptr() for i in range(len(specs))], dtype=np.uint64)[sid] + \
        (slot * n).astype(np.uint64)
    op = np.array([o.data_ptr() for o in outs], dtype=np.uint64)[sid] + (slot * stride).astype(np.uint64)
    assert len(sid) == 100_000
    lat, em = srv.replay_ptrs(sid, np.zeros(len(sid), np.int64), bp, op, np.full(len(sid), n, np.int64))
    c = srv.counters()
    assert c["completed"] == len(sid)
    assert c["live_records"] == 0
    assert c["live_peak"] <= max_inflight
    assert np.all(lat > 0)
    outs_host = [o.cpu().numpy() for o in outs]
    ys = _served_streams(specs, xs, zip(sid.tolist(), slot.tolist()), outs_host, stride, em)
    drv = Served(srv, gpu, specs, torch.int8)
    for i in range(len(specs)):
        drv.flush(i)
        fy, _ = drv.result(i)
        y = np.concatenate(ys[i] + [fy])
        assert len(y) == len(yo[i]) and np.array_equal(y, yo[i]), f"stream {i}"
    srv.close()


@pytest.mark.gpu
def test_ticket_records_bounded_poll_loop(gpu):
    """A submit/poll loop (2 x 10^4 blocks; the client keeps at most
    max_inflight tickets outstanding and polls the oldest to completion
    before submitting more): polled records retire, so the live count
    stays within the in-flight limit; retired tickets report done with
    unknown counts; the output equals the oracle's."""
    specs = [synth.StreamSpec(0, W, 3.0, m, 12.0, 0.01, 8, 200) for W, m in [(4096, 1), (1000, 2)]]
    nblk, n = 10_000, 3008
    for s in specs:
        s.length = nblk * n
    xs = make_streams(specs, SEED + 7)
    yo, _ = oracle_streams(xs, specs, SEED + 7)
    max_inflight = 32
    srv = rfi.Server(elem_size=1, max_streams=2, max_inflight=max_inflight, max_batch=8,
                     hbm_budget_bytes=1 << 32, seed=SEED + 7, n_lanes=1)
    for i, s in enumerate(specs):
        srv.add_stream(i, s.window, s.k, s.mode)
    xd = [torch.from_numpy(x).to(gpu) for x in xs]
    stride = (n + 4096 - 1 + 15) // 16 * 16
    outs = [torch.full((nblk * stride,), 0x5A, dtype=torch.int8, device=gpu) for _ in specs]
    queue, emitted, peak = [], {}, 0
    first = None
    for b in range(nblk):
        for i in range(2):
            blk = xd[i][b * n:(b + 1) * n]
            out = outs[i][b * stride:(b + 1) * stride]
            while True:
                t = srv.try_submit(i, blk, out, None, n=n) if len(queue) < max_inflight else None
                if t is not None:
                    break
                t0, i0, b0 = queue.pop(0)
                while True:
                    done, se, _ = srv.poll(t0)
                    if done:
                        break
                emitted[(i0, b0)] = se
            first = first or t
            queue.append((t, i, b))
            peak = max(peak, srv.counters()["live_records"])
    srv.sync()
    for t, i, b in queue:
        done, se, _ = srv.poll(t)
        assert done
        emitted[(i, b)] = se
    assert peak <= max_inflight
    assert srv.counters()["live_peak"] <= max_inflight
    # the first ticket was polled long ago: retired, done with unknown counts
    assert srv.poll(first) == (True, -1, -1)
    assert srv.ticket_times(first) == (-1, -1)
    with pytest.raises(rfi.RfiError):
        srv.poll(10 ** 9)
    drv = Served(srv, gpu, specs, torch.int8)
    for i in range(2):
        oh = outs[i].cpu().numpy()
        parts = [oh[b * stride:b * stride + emitted[(i, b)]] for b in range(nblk)]
        drv.flush(i)
        fy, _ = drv.result(i)
        y = np.concatenate(parts + [fy])
        assert len(y) == len(yo[i]) and np.array_equal(y, yo[i]), f"stream {i}"
    srv.close()


@pytest.mark.gpu
def test_failed_table_upload_is_undone(gpu, monkeypatch):
    """Table uploads 3 and 4 fail (the server's testing hook): the batch
    built for the third block is undone, its block stays queued, dispatch
    reports the failure, and the next dispatch runs it from the restored
    carry: every output equals the oracle's."""
    specs = [synth.StreamSpec(0, W, 3.0, m, 10.0, 0.01, 8, 200) for W, m in [(4096, 2), (1000, 1)]]
    sizes = [5000, 7000, 3001, 9000, 4096, 1]
    for s in specs:
        s.length = sum(sizes)
    xs = make_streams(specs, SEED + 8)
    yo, sto = oracle_streams(xs, specs, SEED + 8)
    monkeypatch.setenv("RFI_SERVE_FAIL_UPLOAD", "3:2")
    srv = rfi.Server(elem_size=1, max_streams=2, max_inflight=64, max_batch=64,
                     hbm_budget_bytes=1 << 32, seed=SEED + 8, n_lanes=1)
    monkeypatch.delenv("RFI_SERVE_FAIL_UPLOAD")
    for i, s in enumerate(specs):
        srv.add_stream(i, s.window, s.k, s.mode)
    drv = Served(srv, gpu, specs, torch.int8)
    pos = 0
    for j, n in enumerate(sizes):
        for i in range(2):
            t = drv.submit(i, xs[i][pos:pos + n])
            if j == 1 and i == 0:
                # uploads so far: block 0 of each stream (1, 2, each synced);
                # this block's batch is the third: undone, the block queued
                with pytest.raises(rfi.RfiError) as e:
                    srv.dispatch()  # the fourth upload fails too
                assert e.value.status == -4
                assert srv.counters()["completed"] == 2
                srv.poll(t)  # the fifth succeeds
            srv.sync()
        pos += n
    drv.collect()
    for i in range(2):
        drv.flush(i)
        y, st = drv.result(i)
        assert_same(y, st, yo[i], sto[i], f"stream {i}")
    srv.close()
