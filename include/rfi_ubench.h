/*
 * rfi_ubench.h -- microbenchmark kernels shipped with librfimad.
 *
 * rfi_ubench_copy: a plain device-to-device copy used to measure the HBM
 * streaming ceiling of the GPU (the denominator next to the 8 TB/s peak) and
 * to calibrate the FETCH_SIZE / WRITE_SIZE hardware counters against a
 * kernel whose traffic is known (one read and one write per byte).
 *   x, y     device pointers, 16-byte aligned, non-overlapping.
 *   bytes    multiple of 16384.
 *   variant  0: 64 bytes per lane as four 16-byte loads (the tile shape of
 *               the filter kernels), one workgroup per 16 KiB;
 *            1: as 0 with non-temporal loads and stores;
 *            2: 16 bytes per lane, grid-stride loop over a persistent grid;
 *            3: as 1, but each lane's 64 bytes contiguous (the four loads
 *               of a lane 16 bytes apart);
 *            4: as 1, lanes 8g..8g+7 (mod 32) taking their loads in the
 *               rotated order (t + g) mod 4.
 *   stream   hipStream_t (NULL = null stream).
 * Returns 0, RFI_ERR_INVALID (-1) or RFI_ERR_ALIGN (-2); asynchronous.
 *
 * rfi_ubench_lds_hist: the LDS atomic rate of the int8 selection's
 * histogram, the filter's second roof after HBM.  Each workgroup reads a
 * 16 KiB tile of x in the filter's load shape and counts every byte into
 * per-wave LDS histograms of `replicas` copies (replica = lane % replicas),
 * one LDS atomic per byte; the counts of workgroup g are then added to row
 * g % 256 of hist_out.
 *   x          device, 16-byte aligned, bytes a multiple of 16384; bins are
 *              raw byte values 0..255.
 *   replicas   1, 2, 4 or 8.
 *   hist_out   device uint32[256 * 256] (row-major, 256 rows of 256 bins),
 *              4-byte aligned, accumulated into (the caller clears it
 *              first); the byte counts are the column sums.
 * Returns 0, RFI_ERR_INVALID (-1), RFI_ERR_ALIGN (-2) or RFI_ERR_HIP (-5);
 * asynchronous on stream.
 */
#ifndef RFI_UBENCH_H
#define RFI_UBENCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int rfi_ubench_copy(const void* x, void* y, uint64_t bytes, int32_t variant, void* stream);
int rfi_ubench_lds_hist(const void* x, uint64_t bytes, int32_t replicas, uint32_t* hist_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
