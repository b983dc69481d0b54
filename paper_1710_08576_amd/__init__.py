"""rfimad: MI355X-native windowed median/MAD broadband RFI excision.

Per non-overlapping window of each antenna time series: exact (lower)
median, median absolute deviation, the binary32 threshold
t = k * 1.4826 * MAD, and replacement of every sample with |x - m| > t by
zero, by the threshold about the median, or by Philox-driven digital noise
(Buch et al., Sec. II-D, Eqs. (1)-(2)).  All work runs in librfimad.so
(HIP, gfx950); this package is the ctypes binding plus the synthetic-input
generator used by tests and benchmarks.
"""
from ._lib import (  # noqa: F401
    CLIP, NOISE, ZERO, SCHEDULES, STATS_DTYPE, Plan, RfiError, Server, block_power, improvement, layout, load,
    mad_filter, mad_filter_multi, mad_filter_noalloc, mom_filter, mom_filter_carry, n_blocks, stats_numpy, tune_load, tune_save, validate,
)
