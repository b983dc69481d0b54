"""CPU oracle for windowed median/MAD RFI excision -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path (the HIP library and its Python
binding) never does, and shares no code with it.

The arithmetic lives in ``rfi_oracle.c`` (plain C, full sort per window);
this module only builds it with gcc and marshals numpy arrays through ctypes.
Paper: Buch et al., "Implementing and Characterizing Real-time Broadband RFI
Excision for the GMRT Wideband Backend", Sec. II-D, Eqs. (1)-(3); the
improvement metric of Sec. III-A (block power, the ratio S, improvement
in dB) is plain numpy at the end of this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rfi_oracle.c")
_LIB = os.path.join(_HERE, "librfi_oracle.so")

ZERO, CLIP, NOISE = 0, 1, 2

STATS_DTYPE = np.dtype(
    [("median", "<i4"), ("mad", "<i4"), ("n_flagged", "<u4"), ("threshold", "<f4")]
)


def build() -> str:
    """Compile the oracle with gcc (binary32 on SSE, no contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def default_threads() -> int:
    """Host threads for the batch calls: all cores, at most 16 (a host
    shared by several GPUs grants a process one GPU's share of its CPUs,
    whatever the core count shows)."""
    return max(1, min(os.cpu_count() or 1, 16))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_philox4x64_10.restype = None
        L.orc_q8_table.argtypes = [P]
        L.orc_q8_table.restype = None
        L.orc_layout.argtypes = [ctypes.c_int32, P, P, P, P]
        L.orc_layout.restype = ctypes.c_int64
        for name in ("orc_window_i8", "orc_window_i16"):
            f = getattr(L, name)
            f.argtypes = [P, P, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                          ctypes.c_uint64, ctypes.c_float, ctypes.c_int32, P]
            f.restype = None
        for name in ("orc_filter_i8", "orc_filter_i16"):
            f = getattr(L, name)
            f.argtypes = [P, P, ctypes.c_int32, P, P, P, P, ctypes.c_uint64, P,
                          ctypes.c_int32]
            f.restype = ctypes.c_int
        L.orc_mom_filter_i8.argtypes = [P, P, ctypes.c_int32, P, P, P, P, ctypes.c_int32,
                                        ctypes.c_uint64, P, ctypes.c_int32]
        L.orc_mom_filter_i8.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x64_10(ctr, key) -> list[int]:
    """One Philox4x64-10 block for a 4-word counter and a 2-word key."""
    c = np.array([int(v) for v in ctr], dtype=np.uint64)
    k = np.array([int(v) for v in key], dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(v) for v in out]


def q8_table() -> np.ndarray:
    out = np.zeros(4096, dtype=np.int16)
    lib().orc_q8_table(_ptr(out))
    return out


def layout(lengths, windows):
    """(sample_offsets, window_offsets, total_windows) of the packed layout."""
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W = np.ascontiguousarray(windows, dtype=np.int32)
    so = np.zeros(len(L), dtype=np.int64)
    wo = np.zeros(len(L), dtype=np.int64)
    total = lib().orc_layout(len(L), _ptr(L), _ptr(W), _ptr(so), _ptr(wo))
    return so, wo, int(total)


def window(x, k: float, mode: int, *, abs_start: int = 0, stream: int = 0, seed: int = 0):
    """Filter one window; returns (y, stats) with stats a STATS_DTYPE scalar record."""
    x = np.ascontiguousarray(x)
    if x.dtype == np.int8:
        f = lib().orc_window_i8
    elif x.dtype == np.int16:
        f = lib().orc_window_i16
    else:
        raise TypeError("oracle windows are int8 or int16")
    y = np.empty_like(x)
    st = np.zeros(1, dtype=STATS_DTYPE)
    f(_ptr(x), _ptr(y), len(x), abs_start, stream, seed, float(k), int(mode), _ptr(st))
    return y, st[0]


def filter_batch(x, lengths, windows, k, mode, seed: int = 0, n_threads: int | None = None):
    """Whole packed batch; returns (y, stats[total_windows]).

    Padding elements of y (between streams) are copied from x, as the oracle
    never writes them.
    """
    x = np.ascontiguousarray(x)
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W = np.ascontiguousarray(windows, dtype=np.int32)
    K = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.float32), (n,)))
    M = np.ascontiguousarray(np.broadcast_to(np.asarray(mode, dtype=np.int32), (n,)))
    _, _, total = layout(L, W)
    if total < 0:
        raise ValueError("invalid lengths/windows")
    y = x.copy()
    st = np.zeros(max(total, 1), dtype=STATS_DTYPE)
    f = lib().orc_filter_i8 if x.dtype == np.int8 else lib().orc_filter_i16
    if n_threads is None:
        n_threads = default_threads()
    rc = f(_ptr(x), _ptr(y), n, _ptr(L), _ptr(W), _ptr(K), _ptr(M), seed, _ptr(st), n_threads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return y, st[:total]


def mom_filter_batch(x, lengths, windows, k, mode, mom_k: int, seed: int = 0,
                     n_threads: int | None = None):
    """Median-of-MAD filter (Eq. (3)) over a packed int8 batch; returns
    (y, stats[total_windows]).  Padding elements of y are copied from x."""
    x = np.ascontiguousarray(x)
    if x.dtype != np.int8:
        raise TypeError("the median-of-MAD oracle is int8")
    n = len(lengths)
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    W = np.ascontiguousarray(windows, dtype=np.int32)
    K = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.float32), (n,)))
    M = np.ascontiguousarray(np.broadcast_to(np.asarray(mode, dtype=np.int32), (n,)))
    _, _, total = layout(L, W)
    if total < 0:
        raise ValueError("invalid lengths/windows")
    y = x.copy()
    st = np.zeros(max(total, 1), dtype=STATS_DTYPE)
    if n_threads is None:
        n_threads = default_threads()
    rc = lib().orc_mom_filter_i8(_ptr(x), _ptr(y), n, _ptr(L), _ptr(W), _ptr(K), _ptr(M),
                                 int(mom_k), seed, _ptr(st), n_threads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return y, st[:total]


# ---------------------------------------------------------------------------
# Improvement metric (Sec. III-A): a filter's score in dB is ten times the
# base-10 logarithm of S before filtering (S_U) over S after it (S_F), S being
# a figure relating the mean of the integrated power to its RMS.  Its defining
# source is not available; the reading taken here (per segment, RMS deviation
# over mean, averaged) is stated in s_ratio.  Plain numpy, integers exact,
# ratios fp64.
# ---------------------------------------------------------------------------

def block_power(x, lengths, block: int) -> np.ndarray:
    """Integrated power (Sec. III-A): sum of x^2 over each block of
    ``block`` consecutive samples of each stream of a packed batch (streams at 64-element-aligned offsets, a short
    final block is a block of its own); int64, blocks of stream s first."""
    x = np.asarray(x)
    out = []
    off = 0
    for L in lengths:
        L = int(L)
        s = x[off:off + L].astype(np.int64)
        for b in range(0, L, block):
            v = s[b:b + block]
            out.append(int(np.dot(v, v)))
        off += (L + 63) // 64 * 64
    return np.array(out, dtype=np.int64)


def s_ratio(power, seg: int) -> float:
    """S of Sec. III-A (the paper's "average mean-to-RMS ratio"), read as
    the average, over consecutive segments of ``seg`` values, of the
    segment's RMS deviation about its mean (population form) divided by
    that mean.  This orientation is the one under which the printed
    improvement 10 log10(S_U / S_F) is positive when filtering steadies the
    integrated power; the mean over RMS would make every improvement the
    paper reports negative.  Values after the last whole segment are not
    used; no whole segment gives NaN.  A segment with no deviation gives 0
    (NaN when its mean is 0 too), as IEEE division does."""
    p = np.asarray(power, dtype=np.float64)
    n_seg = len(p) // seg
    if n_seg == 0:
        return float("nan")
    ratios = []
    for i in range(n_seg):
        v = p[i * seg:(i + 1) * seg]
        mu = v.sum() / seg
        rms = np.sqrt(((v - mu) ** 2).sum() / seg)
        with np.errstate(divide="ignore", invalid="ignore"):
            ratios.append(np.float64(rms) / np.float64(mu))
    return float(np.sum(ratios) / n_seg)


def improvement(power_u, power_f, lengths, block: int, seg: int) -> np.ndarray:
    """Improvement metric (Sec. III-A), per stream (S_U, S_F, I): S (see
    s_ratio) of the unfiltered and filtered block powers (whole blocks
    only) and the improvement I = 10 log10(S_U / S_F) in dB, as printed.
    ``power_*`` as from block_power."""
    out = np.zeros((len(lengths), 3), dtype=np.float64)
    off = 0
    for s, L in enumerate(lengths):
        L = int(L)
        nb = (L + block - 1) // block
        full = L // block
        su = s_ratio(np.asarray(power_u)[off:off + full], seg)
        sf = s_ratio(np.asarray(power_f)[off:off + full], seg)
        with np.errstate(divide="ignore", invalid="ignore"):
            out[s] = (su, sf, 10.0 * np.log10(np.float64(su) / np.float64(sf)))
        off += nb
    return out
