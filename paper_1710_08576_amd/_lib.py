"""ctypes binding of librfimad (argument marshalling only).

Every filtering step runs in the HIP library; this module only turns torch
tensors into pointers and Python sequences into host arrays.  There is no
fallback: if the library or a HIP device is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfimad.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "rfi_mad.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(_HERE), "include", "rfi_ubench.h")]

RFI_OK = 0
STATUS = {0: "RFI_OK", -1: "RFI_ERR_INVALID", -2: "RFI_ERR_ALIGN", -3: "RFI_ERR_UNSUPPORTED",
          -4: "RFI_ERR_NOMEM", -5: "RFI_ERR_HIP", -6: "RFI_ERR_BUSY"}
ZERO, CLIP, NOISE = 0, 1, 2
(SCHED_AUTO, SCHED_SPLIT, SCHED_SPLIT_PERSIST, SCHED_FUSED, SCHED_PER_STREAM, SCHED_FUSED_PERSIST,
 SCHED_SPLIT_CONCURRENT, SCHED_FUSED_CONCURRENT, SCHED_ONE_LAUNCH, SCHED_ONE_LAUNCH_PERSIST) = range(10)
SCHEDULES = {"auto": 0, "split": 1, "split_persist": 2, "fused": 3, "per_stream": 4,
             "fused_persist": 5, "split_concurrent": 6, "fused_concurrent": 7, "one_launch": 8,
             "one_launch_persist": 9}

STATS_DTYPE = np.dtype(
    [("median", "<i4"), ("mad", "<i4"), ("n_flagged", "<u4"), ("threshold", "<f4")]
)


class RfiError(RuntimeError):
    def __init__(self, status: int, where: str, text: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({text})")


class ServerConfig(ctypes.Structure):
    _fields_ = [("elem_size", ctypes.c_int32), ("max_streams", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("n_lanes", ctypes.c_int32), ("schedule", ctypes.c_int32)]


_lib = None
P = ctypes.c_void_p
I32, I64, U32, U64, F32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "rfi_mad_filter": (ctypes.c_int, [P, P, I32, P, P, P, P, U64, P, P]),
    "rfi_mad_filter_i16": (ctypes.c_int, [P, P, I32, P, P, P, P, U64, P, P]),
    "rfi_mad_filter_noalloc": (ctypes.c_int, [P, P, I32, P, P, P, P, U64, P, P]),
    "rfi_mom_filter": (ctypes.c_int, [P, P, I32, P, P, P, P, I32, U64, P, P]),
    "rfi_mom_filter_carry": (ctypes.c_int, [P, P, I32, P, P, P, P, I32, U64, P, P, P, P, P]),
    "rfi_mad_filter_multi": (ctypes.c_int, [P, I32, P, I32, P, P, P, P, U64, P, P]),
    "rfi_block_power": (ctypes.c_int, [P, I32, I32, P, I32, P, P]),
    "rfi_improvement": (ctypes.c_int, [P, P, I32, P, I32, I32, P, P]),
    "rfi_layout": (ctypes.c_int64, [I32, P, P, P, P, P]),
    "rfi_validate": (ctypes.c_int, [I32, P, P, I32, P, P, P, P, P]),
    "rfi_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rfi_version": (ctypes.c_char_p, []),
    "rfi_plan_create": (ctypes.c_int, [I32, I32, P, P, P, P, U64, PP]),
    "rfi_plan_set_schedule": (ctypes.c_int, [P, I32]),
    "rfi_plan_get_schedule": (ctypes.c_int, [P]),
    "rfi_plan_set_graph": (ctypes.c_int, [P, I32]),
    "rfi_plan_set_option": (ctypes.c_int, [P, I32, I32]),
    "rfi_plan_execute": (ctypes.c_int, [P, P, P, P, P]),
    "rfi_plan_info": (ctypes.c_int, [P, P, P, P, P]),
    "rfi_plan_autotune": (ctypes.c_int, [P, P, P, P, P, I32, P, P]),
    "rfi_plan_destroy": (ctypes.c_int, [P]),
    "rfi_shutdown": (ctypes.c_int, []),
    "rfi_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "rfi_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "rfi_server_create": (ctypes.c_int, [P, PP]),
    "rfi_server_add_stream": (ctypes.c_int, [P, U32, I32, F32, I32]),
    "rfi_server_submit": (ctypes.c_int, [P, U32, P, P, I64, P, P]),
    "rfi_server_dispatch": (ctypes.c_int, [P]),
    "rfi_server_poll": (ctypes.c_int, [P, U64, P, P, P]),
    "rfi_server_sync": (ctypes.c_int, [P]),
    "rfi_server_flush": (ctypes.c_int, [P, U32, P, P, P]),
    "rfi_server_snapshot": (ctypes.c_int, [P, U32, P, P, P]),
    "rfi_server_restore": (ctypes.c_int, [P, U32, I64, I32, P]),
    "rfi_server_counters": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "rfi_server_ticket_times": (ctypes.c_int, [P, U64, P, P]),
    "rfi_server_replay": (ctypes.c_int, [P, I64, P, P, P, P, P, P, P, P]),
    "rfi_server_destroy": (ctypes.c_int, [P]),
    "rfi_ubench_copy": (ctypes.c_int, [P, P, U64, I32, P]),
    "rfi_ubench_lds_hist": (ctypes.c_int, [P, U64, I32, P, P]),
}


def header_symbols() -> list[str]:
    """Every function the public headers declare."""
    names = set()
    for h in HEADERS:
        text = open(h).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(rfi_\w+)\s*\(", text, re.M))
    return sorted(names)


def load():
    """Load librfimad.so (built by build.py).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librfimad.so not built ({LIB_PATH}); run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, where: str):
    if rc != RFI_OK:
        text = load().rfi_status_string(rc)
        raise RfiError(rc, where, text.decode() if text else "")


def _arr(values, dtype, n):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(values, dtype=dtype), (n,)))
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def layout(lengths, windows):
    """(sample_offsets, window_offsets, total_windows, total_elems)."""
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W = _arr(windows, np.int32, len(L))
    so = np.zeros(len(L), dtype=np.int64)
    wo = np.zeros(len(L), dtype=np.int64)
    tot = np.zeros(1, dtype=np.int64)
    nw = load().rfi_layout(len(L), _ptr(L), _ptr(W), _ptr(so), _ptr(wo), _ptr(tot))
    if nw < 0:
        _check(int(nw), "rfi_layout")
    return so, wo, int(nw), int(tot[0])


def validate(elem_size, x_ptr, y_ptr, lengths, windows, k, mode, stats_ptr=0) -> int:
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W, K, M = _arr(windows, np.int32, n), _arr(k, np.float32, n), _arr(mode, np.int32, n)
    return load().rfi_validate(elem_size, P(x_ptr), P(y_ptr), n, _ptr(L), _ptr(W), _ptr(K),
                               _ptr(M), P(stats_ptr))


def ubench_copy(x, y, variant=0, stream=None):
    """HBM copy microbenchmark kernel: y[:] = x[:] (bytes a multiple of 16 KiB)."""
    nbytes = x.numel() * x.element_size()
    _check(load().rfi_ubench_copy(_tptr(x), _tptr(y), nbytes, variant, _stream_handle(stream)),
           "rfi_ubench_copy")


def ubench_lds_hist(x, replicas=4, hist=None, stream=None):
    """LDS histogram-rate microbenchmark: counts the bytes of x (a multiple
    of 16 KiB) into per-wave LDS histograms with `replicas` copies; returns
    the int32 [256, 256] tensor (uint32 counts) it added to, whose column
    sums are the 256 raw-byte counts."""
    import torch
    nbytes = x.numel() * x.element_size()
    if hist is None:
        hist = torch.zeros((256, 256), dtype=torch.int32, device=x.device)
    _check(load().rfi_ubench_lds_hist(_tptr(x), nbytes, int(replicas), _tptr(hist), _stream_handle(stream)),
           "rfi_ubench_lds_hist")
    return hist


def tune_save(path: str):
    """Write the autotune table to a JSON file (rfi_tune_save)."""
    _check(load().rfi_tune_save(os.fsencode(path)), "rfi_tune_save")


def tune_load(path: str):
    """Add the entries of a saved autotune table (rfi_tune_load)."""
    _check(load().rfi_tune_load(os.fsencode(path)), "rfi_tune_load")


def stats_numpy(stats_t) -> np.ndarray:
    """Device stats tensor (int32 [n, 4]) -> numpy structured array."""
    raw = stats_t.detach().cpu().contiguous().numpy()
    return raw.view(STATS_DTYPE).reshape(-1)


def mad_filter(x, lengths, windows, k, mode, seed: int = 0, y=None, stats=True, stream=None):
    """Filter packed streams on the device.  x: int8 or int16 CUDA tensor in
    the packed layout; returns (y, stats) with stats an int32 [n_windows, 4]
    tensor (median, mad, n_flagged, threshold bits) or None."""
    import torch
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W, K, M = _arr(windows, np.int32, n), _arr(k, np.float32, n), _arr(mode, np.int32, n)
    _, _, nw, _ = layout(L, W)
    if y is None:
        y = torch.empty_like(x)
    st = torch.empty((max(nw, 1), 4), dtype=torch.int32, device=x.device) if stats else None
    if x.dtype == torch.int8:
        f = load().rfi_mad_filter
    elif x.dtype == torch.int16:
        f = load().rfi_mad_filter_i16
    else:
        raise TypeError("x must be int8 or int16")
    rc = f(_tptr(x), _tptr(y), n, _ptr(L), _ptr(W), _ptr(K), _ptr(M), seed, _tptr(st),
           _stream_handle(stream))
    _check(rc, "rfi_mad_filter")
    return y, (st[:nw] if st is not None else None)


def mad_filter_noalloc(x, lengths, windows, k, mode, seed: int = 0, y=None, stats=None, stream=None):
    """rfi_mad_filter_noalloc: int8 filtering with the library's fixed
    per-device tables (no allocation in the library).  y and stats (int32
    [n_windows, 4]) are caller buffers; when omitted they are allocated
    here, by torch, before the call.  Returns (y, stats)."""
    import torch
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W, K, M = _arr(windows, np.int32, n), _arr(k, np.float32, n), _arr(mode, np.int32, n)
    if x.dtype != torch.int8:
        raise TypeError("x must be int8")
    if y is None:
        y = torch.empty_like(x)
    rc = load().rfi_mad_filter_noalloc(_tptr(x), _tptr(y), n, _ptr(L), _ptr(W), _ptr(K), _ptr(M), seed,
                                       _tptr(stats), _stream_handle(stream))
    _check(rc, "rfi_mad_filter_noalloc")
    return y, stats


def mad_filter_multi(x, lengths, windows, ks, modes, seed: int = 0, ys=None, stats=True, stream=None):
    """Several outputs from one read: ks[o] / modes[o] are output o's per-stream
    (or scalar) k and mode.  Returns (list of y, list of stats)."""
    import torch
    n, n_out = len(lengths), len(ks)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W = _arr(windows, np.int32, n)
    K = np.ascontiguousarray(np.concatenate([_arr(k, np.float32, n) for k in ks]))
    M = np.ascontiguousarray(np.concatenate([_arr(m, np.int32, n) for m in modes]))
    _, _, nw, _ = layout(L, W)
    if x.dtype != torch.int8:
        raise TypeError("x must be int8")
    if ys is None:
        ys = [torch.empty_like(x) for _ in range(n_out)]
    sts = [torch.empty((max(nw, 1), 4), dtype=torch.int32, device=x.device) for _ in range(n_out)] \
        if stats else None
    yp = (ctypes.c_void_p * n_out)(*[y.data_ptr() for y in ys])
    sp = (ctypes.c_void_p * n_out)(*[t.data_ptr() for t in sts]) if sts is not None else None
    rc = load().rfi_mad_filter_multi(_tptr(x), n_out, ctypes.cast(yp, ctypes.c_void_p), n, _ptr(L), _ptr(W),
                                     _ptr(K), _ptr(M), seed,
                                     ctypes.cast(sp, ctypes.c_void_p) if sp is not None else None,
                                     _stream_handle(stream))
    _check(rc, "rfi_mad_filter_multi")
    return ys, ([t[:nw] for t in sts] if sts is not None else None)


def mom_filter(x, lengths, windows, k, mode, mom_k: int, seed: int = 0, y=None, stats=True,
               stream=None):
    """Median-of-MAD filter (Eq. (3)) of packed int8 streams; returns (y, stats)
    like mad_filter."""
    import torch
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W, K, M = _arr(windows, np.int32, n), _arr(k, np.float32, n), _arr(mode, np.int32, n)
    _, _, nw, _ = layout(L, W)
    if x.dtype != torch.int8:
        raise TypeError("x must be int8")
    if y is None:
        y = torch.empty_like(x)
    st = torch.empty((max(nw, 1), 4), dtype=torch.int32, device=x.device) if stats else None
    rc = load().rfi_mom_filter(_tptr(x), _tptr(y), n, _ptr(L), _ptr(W), _ptr(K), _ptr(M), int(mom_k),
                               seed, _tptr(st), _stream_handle(stream))
    _check(rc, "rfi_mom_filter")
    return y, (st[:nw] if st is not None else None)


def mom_filter_carry(x, lengths, windows, k, mode, mom_k: int, abs_base, history, history_len, seed: int = 0,
                     y=None, stats=True, stream=None):
    """Median-of-MAD filter carried across calls: abs_base (int64 [n]),
    history (uint8 [n, mom_k - 1]) and history_len (int32 [n]) are CUDA
    tensors; history and history_len are updated in place."""
    import torch
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W, K, M = _arr(windows, np.int32, n), _arr(k, np.float32, n), _arr(mode, np.int32, n)
    _, _, nw, _ = layout(L, W)
    if x.dtype != torch.int8:
        raise TypeError("x must be int8")
    if y is None:
        y = torch.empty_like(x)
    st = torch.empty((max(nw, 1), 4), dtype=torch.int32, device=x.device) if stats else None
    rc = load().rfi_mom_filter_carry(_tptr(x), _tptr(y), n, _ptr(L), _ptr(W), _ptr(K), _ptr(M), int(mom_k), seed,
                                     _tptr(abs_base), _tptr(history), _tptr(history_len), _tptr(st),
                                     _stream_handle(stream))
    _check(rc, "rfi_mom_filter_carry")
    return y, (st[:nw] if st is not None else None)


class Plan:
    """A reusable work table for one argument signature."""

    def __init__(self, elem_size, lengths, windows, k, mode, seed=0):
        n = len(lengths)
        self.L = np.ascontiguousarray(lengths, dtype=np.int64)
        self.W = _arr(windows, np.int32, n)
        self.K = _arr(k, np.float32, n)
        self.M = _arr(mode, np.int32, n)
        self.elem_size = elem_size
        self.n_windows = layout(self.L, self.W)[2]
        h = ctypes.c_void_p()
        _check(load().rfi_plan_create(elem_size, n, _ptr(self.L), _ptr(self.W), _ptr(self.K),
                                      _ptr(self.M), seed, ctypes.byref(h)), "rfi_plan_create")
        self.h = h

    def set_schedule(self, sched):
        if isinstance(sched, str):
            sched = SCHEDULES[sched]
        _check(load().rfi_plan_set_schedule(self.h, int(sched)), "rfi_plan_set_schedule")

    def schedule(self) -> int:
        return load().rfi_plan_get_schedule(self.h)

    def set_tiles_per_wg(self, tpw: int):
        _check(load().rfi_plan_set_option(self.h, 1, int(tpw)), "rfi_plan_set_option")

    def set_wg_per_cu(self, n: int):
        _check(load().rfi_plan_set_option(self.h, 2, int(n)), "rfi_plan_set_option")

    def set_graph(self, on: bool):
        _check(load().rfi_plan_set_graph(self.h, 1 if on else 0), "rfi_plan_set_graph")

    def execute(self, x, y, stats=None, stream=None):
        _check(load().rfi_plan_execute(self.h, _tptr(x), _tptr(y), _tptr(stats),
                                       _stream_handle(stream)), "rfi_plan_execute")

    def info(self):
        nl = np.zeros(1, np.int32)
        a = np.zeros(3, np.int64)
        _check(load().rfi_plan_info(self.h, _ptr(nl), _ptr(a[0:1]), _ptr(a[1:2]), _ptr(a[2:3])),
               "rfi_plan_info")
        return {"launches": int(nl[0]), "windows": int(a[0]), "tiles": int(a[1]), "generic": int(a[2])}

    def autotune(self, x, y, stats=None, iters=5, stream=None):
        best = np.zeros(1, np.int32)
        ms = np.zeros(1, np.float32)
        _check(load().rfi_plan_autotune(self.h, _tptr(x), _tptr(y), _tptr(stats),
                                        _stream_handle(stream), iters, _ptr(best), _ptr(ms)),
               "rfi_plan_autotune")
        return int(best[0]), float(ms[0])

    def close(self):
        if getattr(self, "h", None):
            load().rfi_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving runtime: per-stream device carry, admission, batched launches.

    Buffers are CUDA tensors owned by the caller; a block's input, output
    and stats tensors must stay alive until its ticket completes."""

    def __init__(self, elem_size=1, max_streams=64, max_inflight=256, max_batch=64,
                 hbm_budget_bytes=1 << 34, seed=0, n_lanes=2, schedule="fused"):
        if isinstance(schedule, str):
            schedule = SCHEDULES[schedule]
        self.cfg = ServerConfig(elem_size, max_streams, max_inflight, max_batch,
                                hbm_budget_bytes, seed, n_lanes, schedule)
        self.elem_size = elem_size
        self.windows = {}
        h = ctypes.c_void_p()
        _check(load().rfi_server_create(ctypes.byref(self.cfg), ctypes.byref(h)),
               "rfi_server_create")
        self.h = h

    def add_stream(self, sid, window, k, mode):
        _check(load().rfi_server_add_stream(self.h, sid, window, k, mode), "rfi_server_add_stream")
        self.windows[sid] = window

    def out_elems(self, sid, n):
        """Output elements a block of n samples of stream sid needs."""
        return n + self.windows[sid] - 1

    def stats_entries(self, sid, n):
        w = self.windows[sid]
        return (n + w - 1 + w - 1) // w

    def submit(self, sid, block, out, stats=None, n=None) -> int:
        """Returns the ticket; raises RfiError (status RFI_ERR_BUSY) on refusal."""
        if n is None:
            n = block.numel()
        t = ctypes.c_uint64()
        _check(load().rfi_server_submit(self.h, sid, _tptr(block), _tptr(out), n, _tptr(stats),
                                        ctypes.byref(t)), "rfi_server_submit")
        return t.value

    def try_submit(self, sid, block, out, stats=None, n=None):
        """Like submit, but returns None when admission is refused."""
        try:
            return self.submit(sid, block, out, stats, n)
        except RfiError as e:
            if e.status == -6:
                return None
            raise

    def dispatch(self):
        _check(load().rfi_server_dispatch(self.h), "rfi_server_dispatch")

    def poll(self, ticket):
        """(done, samples_emitted, windows_emitted)."""
        d = ctypes.c_int32()
        se, we = ctypes.c_int64(), ctypes.c_int64()
        _check(load().rfi_server_poll(self.h, ticket, ctypes.byref(d), ctypes.byref(se),
                                      ctypes.byref(we)), "rfi_server_poll")
        return bool(d.value), se.value, we.value

    def sync(self):
        _check(load().rfi_server_sync(self.h), "rfi_server_sync")

    def flush(self, sid, out, stats=None) -> int:
        n = ctypes.c_int64()
        _check(load().rfi_server_flush(self.h, sid, _tptr(out), _tptr(stats), ctypes.byref(n)),
               "rfi_server_flush")
        return n.value

    def snapshot(self, sid):
        """(next_index, carry samples as a numpy array)."""
        dt = np.int8 if self.elem_size == 1 else np.int16
        buf = np.zeros(max(self.windows[sid], 1), dtype=dt)
        ni, cl = ctypes.c_int64(), ctypes.c_int32()
        _check(load().rfi_server_snapshot(self.h, sid, ctypes.byref(ni), ctypes.byref(cl),
                                          _ptr(buf)), "rfi_server_snapshot")
        return ni.value, buf[:cl.value].copy()

    def restore(self, sid, next_index, carry):
        dt = np.int8 if self.elem_size == 1 else np.int16
        c = np.ascontiguousarray(carry, dtype=dt)
        _check(load().rfi_server_restore(self.h, sid, next_index, len(c),
                                         _ptr(c) if len(c) else None), "rfi_server_restore")

    def counters(self):
        v = [ctypes.c_uint64() for _ in range(6)]
        _check(load().rfi_server_counters(self.h, *[ctypes.byref(x) for x in v]),
               "rfi_server_counters")
        return dict(zip(("admitted", "refused", "completed", "launches", "live_records", "live_peak"),
                        (x.value for x in v)))

    def ticket_times(self, ticket):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load().rfi_server_ticket_times(self.h, ticket, ctypes.byref(a), ctypes.byref(b)),
               "rfi_server_ticket_times")
        return a.value, b.value

    def replay(self, stream_ids, arrival_ns, blocks, outs, stats=None):
        """Real-time replay (see rfi_server_replay); returns (latency_ns,
        samples_emitted) numpy arrays."""
        n = len(stream_ids)
        sid = np.ascontiguousarray(stream_ids, dtype=np.uint32)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        bp = np.array([b.data_ptr() for b in blocks], dtype=np.uint64)
        op = np.array([o.data_ptr() for o in outs], dtype=np.uint64)
        ln = np.array([b.numel() for b in blocks], dtype=np.int64)
        sp = np.array([s.data_ptr() for s in stats], dtype=np.uint64) if stats is not None else None
        lat = np.zeros(n, np.int64)
        em = np.zeros(n, np.int64)
        _check(load().rfi_server_replay(self.h, n, _ptr(sid), _ptr(arr), _ptr(bp), _ptr(op),
                                        _ptr(ln), _ptr(sp) if sp is not None else None,
                                        _ptr(lat), _ptr(em)), "rfi_server_replay")
        return lat, em

    def replay_ptrs(self, stream_ids, arrival_ns, block_ptrs, out_ptrs, lengths, stats_ptrs=None):
        """replay() on raw device addresses (numpy uint64 arrays)."""
        n = len(stream_ids)
        sid = np.ascontiguousarray(stream_ids, dtype=np.uint32)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        bp = np.ascontiguousarray(block_ptrs, dtype=np.uint64)
        op = np.ascontiguousarray(out_ptrs, dtype=np.uint64)
        ln = np.ascontiguousarray(lengths, dtype=np.int64)
        sp = np.ascontiguousarray(stats_ptrs, dtype=np.uint64) if stats_ptrs is not None else None
        lat = np.zeros(n, np.int64)
        em = np.zeros(n, np.int64)
        _check(load().rfi_server_replay(self.h, n, _ptr(sid), _ptr(arr), _ptr(bp), _ptr(op),
                                        _ptr(ln), _ptr(sp) if sp is not None else None,
                                        _ptr(lat), _ptr(em)), "rfi_server_replay")
        return lat, em

    def close(self):
        if getattr(self, "h", None):
            load().rfi_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def n_blocks(lengths, block: int) -> int:
    """Number of blocks (a short final block counts) over all streams; 0 for
    a block below 1 (the library rejects it)."""
    if block < 1:
        return 0
    return int(sum((int(L) + block - 1) // block for L in lengths))


def block_power(x, lengths, block: int, out=None, stream=None):
    """Sum of x^2 over each block of ``block`` samples of each stream of a
    packed int8/int16 CUDA tensor; returns an int64 tensor, blocks of stream
    0 first (Sec. III-A integrated power)."""
    import torch
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    if x.dtype not in (torch.int8, torch.int16):
        raise TypeError("x must be int8 or int16")
    nb = n_blocks(L, block)
    if out is None:
        out = torch.empty(max(nb, 1), dtype=torch.int64, device=x.device)
    rc = load().rfi_block_power(_tptr(x), x.element_size(), len(L), _ptr(L), int(block), _tptr(out),
                                _stream_handle(stream))
    _check(rc, "rfi_block_power")
    return out[:nb]


def improvement(power_u, power_f, lengths, block: int, seg_blocks: int, out=None, stream=None):
    """Per stream (S_U, S_F, I = 10 log10(S_U / S_F) dB) from unfiltered and
    filtered block powers (Sec. III-A improvement metric; S = average over
    segments of RMS deviation over mean); returns a float64 [n_streams, 3]
    tensor."""
    import torch
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    if out is None:
        out = torch.empty((max(len(L), 1), 3), dtype=torch.float64, device=power_u.device)
    rc = load().rfi_improvement(_tptr(power_u), _tptr(power_f), len(L), _ptr(L), int(block), int(seg_blocks),
                                _tptr(out), _stream_handle(stream))
    _check(rc, "rfi_improvement")
    return out[:len(L)]
