/*
 * rfi_oracle.h -- CPU oracle for windowed median/MAD broadband RFI excision.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no source
 * with the GPU library (no headers, tables, generators or helpers).
 *
 * What it computes (Buch et al., "Implementing and Characterizing Real-time
 * Broadband RFI Excision for the GMRT Wideband Backend", Sec. II-D):
 *   per non-overlapping window of one input's time series, the median M(x),
 *   the median absolute deviation D, the thresholds of Eq. (1)
 *   M(x) +/- n * (1.4826 * D), and the replacement of Eq. (2) for every
 *   sample outside them (by zero, by the threshold, or by digital noise);
 *   and the median-of-MAD variant of Eq. (3), which puts the median of the
 *   MADs of k successive windows in place of D.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - lower median: rank r = floor((N-1)/2) of the sorted window;
 *   - MAD about that median with the same rank;
 *   - threshold t = k * (1.4826f * (float)D), two binary32 multiplies;
 *   - strict comparison |x - m| > t (Eq. (2) as printed is inclusive; the
 *     inclusive form flags every sample of a window with D = 0);
 *   - "threshold" replacement is m +/- floor(t), saturated to the dtype;
 *   - "constant" replacement is 0 (every experiment in Sec. III uses zeros);
 *   - "digital noise" is m + q, q drawn from a Q8 Gaussian quantile table
 *     scaled by the robust sigma, indexed by a 12-bit field of a
 *     Philox4x64-10 block (Salmon et al., SC'11) keyed by (seed, stream):
 *     counter j >> 2 for absolute sample index j, word j & 3, top 12 bits;
 *   - a short final window is a window of its own;
 *   - median of MAD: the k windows are the current one and the k-1 before
 *     it (causal, sliding), fewer at the start of a stream; lower median.
 */
#ifndef RFI_ORACLE_H
#define RFI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t  median;     /* M(x), lower median of the window            */
    int32_t  mad;        /* D, median of |x - M(x)|                     */
    uint32_t n_flagged;  /* number of samples with |x - M(x)| > t       */
    float    threshold;  /* t = k * (1.4826f * D), binary32             */
} orc_stats;

enum { ORC_ZERO = 0, ORC_CLIP = 1, ORC_NOISE = 2 };

/* Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Q8 Gaussian quantile table: G[u] = round(256 * PhiInv((u + 0.5) / 4096)). */
void orc_q8_table(int16_t out[4096]);

/* Packed stream layout: stream s starts at sum_{j<s} align_up(L_j, 64)
 * elements; its windows' stats start at sum_{j<s} ceil(L_j / W_j).
 * Returns the total number of windows, or -1 on a negative length/window. */
int64_t orc_layout(int32_t n_streams, const int64_t* lengths, const int32_t* windows,
                   int64_t* sample_offsets, int64_t* window_offsets);

/* One window of n samples (n >= 1) of stream `stream`, whose first sample
 * has absolute index `abs_start` within that stream.  Writes n outputs to y
 * (y may equal x) and the window's stats to *st (if st is not NULL). */
void orc_window_i8(const int8_t* x, int8_t* y, int32_t n, int64_t abs_start,
                   uint32_t stream, uint64_t seed, float k, int32_t mode, orc_stats* st);
void orc_window_i16(const int16_t* x, int16_t* y, int32_t n, int64_t abs_start,
                    uint32_t stream, uint64_t seed, float k, int32_t mode, orc_stats* st);

/* Whole batch in the packed layout above, windows spread over n_threads
 * POSIX threads (n_threads <= 0 means 1).  stats may be NULL.
 * Returns 0, or -1 on an invalid argument. */
int orc_filter_i8(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                  const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                  orc_stats* stats, int32_t n_threads);
int orc_filter_i16(const int16_t* x, int16_t* y, int32_t n_streams, const int64_t* lengths,
                   const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                   orc_stats* stats, int32_t n_threads);

/* Median of MAD (Eq. (3)), int8.  Per stream: the lower median M(x) and
 * MAD D of every window as above; for window w the threshold uses
 * M_m(w) = lower median of the MADs of windows max(0, w-K+1) .. w
 * (K = mom_k >= 1; fewer at the start of the stream) in place of D:
 * t = k * (1.4826f * (float)M_m(w)), flag |x - M(x)| > t, replacement and
 * noise scale as above with M_m(w).  Stats: median, the window's own MAD,
 * n_flagged, t.  Streams are spread over n_threads threads.
 * Returns 0, or -1 on an invalid argument. */
int orc_mom_filter_i8(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                      const int32_t* windows, const float* k, const int32_t* mode, int32_t mom_k,
                      uint64_t seed, orc_stats* stats, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
