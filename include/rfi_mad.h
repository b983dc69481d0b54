/*
 * rfi_mad.h -- C ABI of librfimad, MI355X (gfx950) windowed median/MAD
 * broadband RFI excision.
 *
 * The method (Buch et al., "Implementing and Characterizing Real-time
 * Broadband RFI Excision for the GMRT Wideband Backend", Sec. II-D):
 * each input's time series is cut into non-overlapping windows; per window
 * the median M(x) and the median absolute deviation D are found, the
 * thresholds of Eq. (1) are M(x) +/- n * (1.4826 * D) (the multiple n is the
 * argument `k` here), and Eq. (2) replaces every sample outside them.
 *
 * Conventions fixed by this library (where the paper is silent):
 *   - windows are contiguous, aligned at sample 0 of each stream, and a
 *     short final window is a window of its own;
 *   - median = lower median, the sample of rank floor((N-1)/2) in sorted
 *     order; MAD = the same rank of |x - median|;
 *   - t = k * (1.4826f * (float)D), two IEEE binary32 round-to-nearest
 *     multiplies; a sample is flagged iff |x - median| > t (strict);
 *   - replacements (`mode`):
 *       RFI_MODE_ZERO   0
 *       RFI_MODE_CLIP   median +/- floor(t) on the sample's side, saturated
 *       RFI_MODE_NOISE  saturate(median + q), q = (s * G[u] + 2^15) >> 16
 *                       (arithmetic shift), s = (int)(1.4826f*D * 256.0f),
 *                       G[u] = round(256 * PhiInv((u + 0.5) / 4096)),
 *                       u = the 12 most significant bits of word j & 3
 *                       of the Philox4x64-10 block (Salmon et al.,
 *                       SC'11) with key (seed, stream) and counter
 *                       (j >> 2, 0, 0, 0): one block per 4 samples;
 *                       j = absolute sample index within the stream.
 *   - statistics are taken from the input window in every mode.
 *
 * Packed layout used by every batch entry point:
 *   stream s occupies elements [off_s, off_s + L_s) of x and y, with
 *   off_s = sum_{j<s} align_up(L_j, 64); the buffers must hold at least
 *   off_{n-1} + align_up(L_{n-1}, 64) elements.  Elements between streams
 *   (padding) are read but never written.  Window w of stream s writes
 *   stats[woff_s + w], woff_s = sum_{j<s} ceil(L_j / W_j).  rfi_layout()
 *   computes both offset arrays.
 *
 * Ownership and threading: x, y, stats are caller-owned device memory that
 * must stay valid until the enqueued work has run on `stream`; the host
 * arrays (lengths, windows, k, mode) are read during the call only.  All
 * work is asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 * y == x (exactly in place) is allowed; any other overlap is rejected.
 * Errors: every entry point returns an rfi_status.  Argument errors
 * (RFI_ERR_INVALID, RFI_ERR_ALIGN, RFI_ERR_UNSUPPORTED) are found before
 * anything is enqueued; after RFI_ERR_NOMEM or RFI_ERR_HIP from a call that
 * runs several passes, earlier passes may already be enqueued and the
 * outputs are undefined.  Device faults surface at the caller's
 * synchronisation.
 */
#ifndef RFI_MAD_H
#define RFI_MAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RFI_OK = 0,
    RFI_ERR_INVALID = -1,     /* bad argument value or size                  */
    RFI_ERR_ALIGN = -2,       /* x, y or stats not 16-byte aligned           */
    RFI_ERR_UNSUPPORTED = -3, /* valid request the library cannot serve     */
    RFI_ERR_NOMEM = -4,       /* device or host allocation failed            */
    RFI_ERR_HIP = -5,         /* a HIP runtime call failed (see status text) */
    RFI_ERR_BUSY = -6         /* serving: admission refused (budget/slots)   */
} rfi_status;

typedef enum { RFI_MODE_ZERO = 0, RFI_MODE_CLIP = 1, RFI_MODE_NOISE = 2 } rfi_mode;

/* Per-window statistics, 16 bytes, computed from the input window. */
typedef struct {
    int32_t median;     /* lower median M(x)                          */
    int32_t mad;        /* D = median |x - M(x)|                      */
    uint32_t n_flagged; /* samples with |x - M(x)| > threshold        */
    float threshold;    /* t = k * (1.4826f * D), binary32            */
} rfi_window_stats;

/* Limits checked by rfi_validate. */
#define RFI_MAX_WINDOW 65536
#define RFI_MAX_K 1.0e4f
#define RFI_MAX_BLOCK (1 << 30) /* rfi_block_power, rfi_improvement */

/* ------------------------------------------------------------------ */
/* Batch filtering (Sec. II-D, Eqs. (1)-(2)).                          */
/* ------------------------------------------------------------------ */

/* Filter n_streams packed int8 streams.
 *   x, y      device pointers, 16-byte aligned, packed layout above.
 *   lengths   host array [n_streams], L_s >= 0 samples.
 *   windows   host array [n_streams], 1 <= W_s <= RFI_MAX_WINDOW.
 *   k         host array [n_streams], finite, 0 <= k <= RFI_MAX_K.
 *   mode      host array [n_streams], rfi_mode values.
 *   seed      Philox key word 0 for NOISE replacement.
 *   stats_out device pointer [total windows] or NULL (no statistics).
 *   stream    hipStream_t (NULL = null stream).
 * Plans (work tables) are cached per distinct argument signature. */
int rfi_mad_filter(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                   const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                   rfi_window_stats* stats_out, void* stream);

/* Same for int16 samples (radix-select median and MAD). */
int rfi_mad_filter_i16(const int16_t* x, int16_t* y, int32_t n_streams, const int64_t* lengths,
                       const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                       rfi_window_stats* stats_out, void* stream);

/* Layout helper (host only): fills sample_offsets[n] and window_offsets[n]
 * (either may be NULL) and returns the total number of windows, or
 * RFI_ERR_INVALID.  The element count the buffers need is returned in
 * *total_elems when that pointer is not NULL. */
int64_t rfi_layout(int32_t n_streams, const int64_t* lengths, const int32_t* windows,
                   int64_t* sample_offsets, int64_t* window_offsets, int64_t* total_elems);

/* Argument check of rfi_mad_filter[_i16] without touching the device
 * (host only).  elem_size is 1 (int8) or 2 (int16). */
int rfi_validate(int32_t elem_size, const void* x, const void* y, int32_t n_streams,
                 const int64_t* lengths, const int32_t* windows, const float* k,
                 const int32_t* mode, const void* stats_out);

/* Static text for a status code; for RFI_ERR_HIP, the last HIP error seen
 * by this thread. */
const char* rfi_status_string(int status);

/* Integrated power for the improvement metric (Sec. III-A, which scores a
 * filter on integrated power; here it is integrated over blocks of time
 * samples).  For each stream s of a packed batch (the layout above) and
 * each block b of `block` consecutive samples (a short final block is a
 * block of its own): power_out[boff_s + b] = sum of x^2 over the block,
 * exact, with boff_s = sum_{j<s} ceil(L_j / block).
 *   x          device, int8 (elem_bytes 1) or int16 (elem_bytes 2),
 *              16-byte aligned; read only (padding elements are read).
 *   block      1 <= block <= RFI_MAX_BLOCK.
 *   power_out  device int64 [sum_s ceil(L_s / block)], 8-byte aligned,
 *              must not overlap x.
 * Errors: RFI_ERR_INVALID (sizes, NULL with work to do, overlap),
 * RFI_ERR_ALIGN, RFI_ERR_NOMEM, RFI_ERR_HIP.  Asynchronous on `stream`.
 * Blocks of more than 64 KiB are summed in 64 KiB parts (a work buffer of
 * 8 bytes per part is kept by the library per lengths/block signature and
 * stream, so calls on different streams do not share it). */
int rfi_block_power(const void* x, int32_t elem_bytes, int32_t n_streams, const int64_t* lengths,
                    int32_t block, int64_t* power_out, void* stream);

/* Improvement metric (Sec. III-A), which the paper gives in dB as
 * 10 log10(S_U / S_F) of a figure S relating the mean of the integrated
 * power to its RMS, unfiltered (U) and filtered (F).  Inputs are the block
 * powers of an unfiltered (power_u) and a filtered (power_f) batch, both
 * laid out as rfi_block_power writes them for the same lengths and block.
 * Per stream, over its whole blocks only (a short final block is not used):
 * the values are cut into floor(whole_blocks / seg_blocks) segments of
 * seg_blocks consecutive blocks (the rest is not used); S is the average
 * over segments of the segment's population RMS deviation about its mean
 * divided by that mean.  out[3 s + 0] = S_U, out[3 s + 1] = S_F,
 * out[3 s + 2] = 10 log10(S_U / S_F) in dB (positive when the filtered
 * power is steadier), binary64 on the device (device buffer, 8-byte
 * aligned).  No whole segment: NaN; a segment without deviation adds 0 to
 * S (IEEE division; 0 / 0 = NaN for an all-zero segment).
 * seg_blocks >= 1.  Errors as rfi_block_power.  Asynchronous on `stream`. */
int rfi_improvement(const int64_t* power_u, const int64_t* power_f, int32_t n_streams, const int64_t* lengths,
                    int32_t block, int32_t seg_blocks, double* out, void* stream);

/* Version string of the library build. */
const char* rfi_version(void);

/* Several outputs from one read, int8: the paper's test arrangement in
 * which one input is copied to several filters with different thresholds
 * and replacement options side by side (Sec. III-A, second test scheme).
 * n_out (1..3) outputs y[0..n_out); output o uses the
 * per-stream arrays k[o * n_streams + s] and mode[o * n_streams + s] and is
 * bit-identical to rfi_mad_filter(x, y[o], ..., that k, that mode, seed,
 * stats_out[o], stream).  stats_out may be NULL, as may any stats_out[o].
 * Outputs must not overlap x or each other (RFI_ERR_INVALID); other
 * arguments and errors as rfi_mad_filter.  The outputs with no noise
 * stream share one read of x for the windows of a tile class (other
 * windows: one read per output); an output with noise streams is computed
 * by a pass of its own. */
int rfi_mad_filter_multi(const int8_t* x, int32_t n_out, int8_t* const* y, int32_t n_streams,
                         const int64_t* lengths, const int32_t* windows, const float* k,
                         const int32_t* mode, uint64_t seed, rfi_window_stats* const* stats_out,
                         void* stream);

/* Median of MAD (Eq. (3)), int8.  Same buffers, layout, ownership,
 * asynchrony and errors as rfi_mad_filter, plus mom_k >= 1 (else
 * RFI_ERR_INVALID).  Each window's threshold uses, in place of its own MAD,
 * the lower median of the MADs of the mom_k windows of its stream ending
 * at it (fewer at the start of the stream):
 *   t = k * (1.4826f * (float)M_m),  M_m = lowmed(D_{w-K+1} .. D_w);
 * the centre stays the window's median, the noise scale is
 * (int)(1.4826f * M_m * 256.0f).  stats_out receives the window's median,
 * its own MAD, the flag count and t (it may be NULL).  Three passes over
 * the batch (statistics, median of MADs, replacement): the input is read
 * twice.  Work tables and temporaries (a few bytes per window) are kept by
 * the library per argument signature and stream, so calls on different
 * streams do not share them; rfi_shutdown frees them. */
int rfi_mom_filter(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                   const int32_t* windows, const float* k, const int32_t* mode, int32_t mom_k,
                   uint64_t seed, rfi_window_stats* stats_out, void* stream);

/* Median of MAD carried across calls, for streams that arrive in pieces
 * (real-time use): as rfi_mom_filter, plus per stream the MADs of its
 * earlier windows and the absolute index of its first sample, so that a
 * stream cut at window boundaries into consecutive calls gives the same
 * output and statistics as one rfi_mom_filter call over the whole stream
 * (a short final window only in the last piece).
 *   abs_base     device int64[n_streams] (8-byte aligned) or NULL (all 0):
 *                absolute index of each stream's first sample in this
 *                call (drives the noise counter).
 *   mad_history  device uint8[n_streams * (mom_k - 1)]: per stream the MADs
 *                of its latest earlier windows, right-aligned (slot
 *                mom_k - 2 holds the most recent), in and out.
 *   history_len  device int32[n_streams] (4-byte aligned): how many slots
 *                hold valid MADs (0 for a new stream, at most mom_k - 1;
 *                clamped to that range), in and out.
 * With mom_k == 1 neither history argument is used (they may be NULL).
 * Errors as rfi_mom_filter; RFI_ERR_INVALID also for NULL history arrays
 * when mom_k > 1.  Work buffers are kept per signature, mom_k and stream. */
int rfi_mom_filter_carry(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                         const int32_t* windows, const float* k, const int32_t* mode, int32_t mom_k,
                         uint64_t seed, const int64_t* abs_base, uint8_t* mad_history, int32_t* history_len,
                         rfi_window_stats* stats_out, void* stream);

/* rfi_mad_filter without allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight real-time loops,
 * harnesses that forbid hipMalloc.  Arguments, layout, results (bit for
 * bit), asynchrony and argument errors are those of rfi_mad_filter.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine, no host-to-device copy): the per-stream descriptors and the
 * work items it would keep in a plan are written by a device kernel into
 * a fixed array of 4 MiB in device memory that each GPU holds from the
 * first call on it until the process ends.
 * Limits (else RFI_ERR_UNSUPPORTED, nothing enqueued):
 *   n_streams <= RFI_NOALLOC_MAX_STREAMS, and at most RFI_NOALLOC_MAX_ITEMS
 *   work items, counted per stream as: W in {512, 1024, 2048, 4096, 8192,
 *   16384}: floor(L / 16384) + ceil(L / W) - floor(L / 16384) * (16384 / W);
 *   any other W: ceil(L / W).
 * Every call on one GPU rewrites that GPU's array: calls that overlap on
 * one GPU (from two host threads, or on two HIP streams the caller does
 * not order) race and give undefined results; calls ordered on one stream,
 * or on different GPUs, do not. */
#define RFI_NOALLOC_MAX_STREAMS 1024
#define RFI_NOALLOC_MAX_ITEMS 257536
int rfi_mad_filter_noalloc(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                           const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                           rfi_window_stats* stats_out, void* stream);

/* ------------------------------------------------------------------ */
/* Explicit plans: a work table for one argument signature, reusable   */
/* across calls, with a selectable launch schedule and HIP-graph       */
/* replay.  rfi_mad_filter uses the same machinery through a cache.    */
/* ------------------------------------------------------------------ */
typedef struct rfi_plan rfi_plan;

typedef enum {
    RFI_SCHED_AUTO = 0,        /* autotuned table, else RFI_SCHED_SPLIT         */
    RFI_SCHED_SPLIT = 1,       /* one launch per window class, one WG per tile  */
    RFI_SCHED_SPLIT_PERSIST = 2, /* one persistent launch per window class     */
    RFI_SCHED_FUSED = 3,       /* one launch for every class, one WG per item   */
    RFI_SCHED_PER_STREAM = 4,  /* one ordinary launch per stream (baseline)     */
    RFI_SCHED_FUSED_PERSIST = 5, /* one persistent launch for every class      */
    RFI_SCHED_SPLIT_CONCURRENT = 6, /* SPLIT's launches spread over four HIP
                                    streams (parallel branches of the graph
                                    when captured), joined on the caller's
                                    stream                                 */
    RFI_SCHED_FUSED_CONCURRENT = 7, /* FUSED's per-mode launches on parallel
                                    streams, joined likewise             */
    RFI_SCHED_ONE_LAUNCH = 8,  /* the whole batch, every class and mode, as
                                  one launch, one WG per item              */
    RFI_SCHED_ONE_LAUNCH_PERSIST = 9, /* the same as one persistent launch */
    RFI_SCHED_COUNT = 10
} rfi_schedule;

/* elem_size 1 or 2; arrays as in rfi_mad_filter.  Allocates device work
 * tables (hipMalloc) and copies them synchronously. */
int rfi_plan_create(int32_t elem_size, int32_t n_streams, const int64_t* lengths,
                    const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                    rfi_plan** out);
int rfi_plan_set_schedule(rfi_plan* plan, int32_t schedule);
int rfi_plan_get_schedule(const rfi_plan* plan);
/* use_graph != 0: capture the launches into a HIP graph on first use with a
 * given (x, y, stats, stream) and replay it afterwards (not on the null
 * stream, where launches are direct). */
int rfi_plan_set_graph(rfi_plan* plan, int32_t use_graph);
int rfi_plan_execute(rfi_plan* plan, const void* x, void* y, rfi_window_stats* stats_out,
                     void* stream);
/* Plan options.
 *   RFI_OPT_TILES_PER_WG  int8 tiles (16 KiB) per workgroup in launches with
 *                         one workgroup per item: 1, 2 (the second tile's
 *                         loads overlap the first tile's work) or 0 (use
 *                         the autotuned value, default 1).
 *   RFI_OPT_WG_PER_CU     at most this many workgroups resident per compute
 *                         unit (1..32, enforced by padding LDS), 0 = no cap,
 *                         -1 = the autotuned value (default; 8 untuned). */
typedef enum { RFI_OPT_TILES_PER_WG = 1, RFI_OPT_WG_PER_CU = 2 } rfi_option;
int rfi_plan_set_option(rfi_plan* plan, int32_t option, int32_t value);
/* Number of kernel launches one execute makes, and total windows. */
int rfi_plan_info(const rfi_plan* plan, int32_t* n_launches, int64_t* n_windows,
                  int64_t* n_tiles, int64_t* n_generic);
/* Time every schedule on the given buffers (iters executes each, median
 * per schedule), select the fastest and report it and its time (ms).
 * Writes y and stats (as one execute would).  y must not be x
 * (RFI_ERR_INVALID): the candidates run repeatedly on the same buffers. */
int rfi_plan_autotune(rfi_plan* plan, const void* x, void* y, rfi_window_stats* stats_out,
                      void* stream, int32_t iters, int32_t* best_schedule, float* best_ms);
int rfi_plan_destroy(rfi_plan* plan);

/* Autotune table persistence.  The table maps (GPU architecture, plan
 * signature: element size, window classes present, irregular windows,
 * noise streams, generic work items) to the chosen schedule, tiles per
 * workgroup and occupancy cap; RFI_SCHED_AUTO plans and the cached batch
 * entry points use it.
 * rfi_tune_save writes every entry of this process's table as JSON
 * ({"entries": [{"arch", "signature" (hex), "schedule" (name), "tiles_per_wg",
 * "wg_per_cu", "ms", and readable signature fields}]}), replacing `path`
 * atomically (a temporary file renamed).  rfi_tune_load adds the entries of
 * such a file (entries of other architectures are kept but match no
 * device here), replacing those of equal keys; a plan built afterwards
 * uses them.  Both are host only.  Errors: RFI_ERR_INVALID (NULL path,
 * file not readable or writable, malformed file: nothing is loaded).
 * With the environment variable RFI_TUNE_FILE set, the library loads that
 * file when it builds its first plan (a missing file is no error) and
 * writes the table to it after every rfi_plan_autotune. */
int rfi_tune_save(const char* path);
int rfi_tune_load(const char* path);

/* Drop cached plans and graphs (all devices of this process). */
int rfi_shutdown(void);

/* ------------------------------------------------------------------ */
/* Serving: blocks of many streams arrive over time, as the digitised  */
/* antenna streams of the paper's real-time backend do (Sec. II-D,     */
/* Sec. III); each stream keeps its carry (the samples of an           */
/* unfinished window) on the device and its absolute sample index on   */
/* the host, so the output equals that of one batch call over the      */
/* concatenated blocks (same windows, same noise draws).  Blocks are   */
/* admitted against an HBM budget and an in-flight limit and filled    */
/* into shared batched launches (continuous batching): stream s runs   */
/* on lane s % n_lanes (one HIP stream each); a lane launches, per     */
/* batch, the next admitted block of each of its streams (at most      */
/* max_batch blocks) as one fused kernel launch plus one carry-update  */
/* launch, and keeps up to two batches in flight.                      */
/* Output of a stream is emitted window by window: a submit emits the  */
/* carry plus as many whole windows as the block completes, into       */
/* out_dev, which must hold n + W - 1 elements.                        */
/* Calls on one server are serialised by a mutex.                     */
/* Ticket records: each admitted block has a record (about 100 bytes)  */
/* until it is retired: a completed ticket once it has been polled     */
/* done (at the next admission after that poll), a completed ticket   */
/* never polled once 65536 later tickets have completed, and the       */
/* tickets of rfi_server_replay as soon as they complete.  At most     */
/* max_inflight + 65536 records are live; a poll-driven loop that      */
/* polls its tickets as they complete keeps about max_inflight.        */
/* Failures: if the work tables of a batch cannot be staged (memory),  */
/* the batch is undone and its blocks wait for the next dispatch (the  */
/* error is returned by dispatch, poll, sync; submit still admits).    */
/* If a kernel launch or a completion query fails, the device state    */
/* of the streams is unknown: the server is faulted and every later    */
/* call except counters and destroy returns RFI_ERR_HIP.               */
/* Testing aid: with the environment variable                          */
/* RFI_SERVE_FAIL_UPLOAD=first[:count] set when a server is created,   */
/* its table uploads number first .. first + count - 1 (counted from   */
/* 1) fail with RFI_ERR_NOMEM, to exercise the undo.                   */
/* ------------------------------------------------------------------ */
typedef struct rfi_server rfi_server;

typedef struct {
    int32_t elem_size;          /* 1 (int8) or 2 (int16)                     */
    int32_t max_streams;        /* stream ids are 0 .. max_streams-1          */
    int32_t max_inflight;       /* blocks admitted but not yet completed      */
    int32_t max_batch;          /* blocks per launch                          */
    uint64_t hbm_budget_bytes;  /* in+out bytes of admitted, unfinished blocks */
    uint64_t seed;              /* Philox key word 0                          */
    int32_t n_lanes;            /* HIP streams used for overlapping batches   */
    int32_t schedule;           /* RFI_SCHED_AUTO or RFI_SCHED_FUSED: one WG  */
                                /* per work item; RFI_SCHED_FUSED_PERSIST: a  */
                                /* grid of resident WGs loops over the items */
} rfi_server_config;

int rfi_server_create(const rfi_server_config* cfg, rfi_server** out);
/* Register stream `stream_id` with its window, threshold multiple and
 * replacement mode (the Philox key word 1 is stream_id). */
int rfi_server_add_stream(rfi_server* srv, uint32_t stream_id, int32_t window, float k,
                          int32_t mode);
/* Admit one block of n samples of stream_id (block_dev: device memory of
 * n elements, 16-byte aligned, valid until the ticket completes).  Output
 * goes to out_dev (n + W - 1 elements), stats of the emitted windows to
 * stats_dev (ceil((n + W - 1) / W) entries, may be NULL).  Returns
 * RFI_ERR_BUSY when the budget or the in-flight limit is reached. */
int rfi_server_submit(rfi_server* srv, uint32_t stream_id, const void* block_dev, void* out_dev,
                      int64_t n, rfi_window_stats* stats_dev, uint64_t* ticket);
/* Launch whatever admitted blocks are not yet on the device (one batched
 * launch per max_batch blocks).  Called by submit when a batch fills. */
int rfi_server_dispatch(rfi_server* srv);
/* done = 1 once the ticket's block has been filtered; samples_emitted and
 * windows_emitted report what its out/stats buffers received.  A retired
 * ticket (see above) reports done = 1 and -1 for both counts; a ticket id
 * never issued is RFI_ERR_INVALID. */
int rfi_server_poll(rfi_server* srv, uint64_t ticket, int32_t* done, int64_t* samples_emitted,
                    int64_t* windows_emitted);
/* Block until every admitted block has completed. */
int rfi_server_sync(rfi_server* srv);
/* End of stream: filter the carry as a short final window into out_dev
 * (W - 1 elements) / stats_dev (1 entry); *n_out receives its length. */
int rfi_server_flush(rfi_server* srv, uint32_t stream_id, void* out_dev,
                     rfi_window_stats* stats_dev, int64_t* n_out);
/* Carry state of one stream, for checkpoint/restore: absolute index of
 * the next sample, carry length, and the carry samples (host buffer of
 * at least W - 1 elements). */
int rfi_server_snapshot(rfi_server* srv, uint32_t stream_id, int64_t* next_index,
                        int32_t* carry_len, void* carry_host);
int rfi_server_restore(rfi_server* srv, uint32_t stream_id, int64_t next_index,
                       int32_t carry_len, const void* carry_host);
/* Counters: admitted, refused (BUSY), completed, launches, ticket
 * records live now and at most so far (any pointer may be NULL). */
int rfi_server_counters(rfi_server* srv, uint64_t* admitted, uint64_t* refused, uint64_t* completed,
                        uint64_t* launches, uint64_t* live_records, uint64_t* live_peak);
/* Host steady-clock times (ns) of a ticket's admission and of the moment
 * the server saw its batch complete (0 while not complete; -1 for both
 * once the ticket is retired). */
int rfi_server_ticket_times(rfi_server* srv, uint64_t ticket, int64_t* t_submit_ns,
                            int64_t* t_done_ns);
/* Real-time replay: block i of stream stream_ids[i] (device buffers
 * blocks[i] / outs[i] / stats[i] as for submit, lengths[i] samples)
 * arrives arrival_ns[i] after the call starts (non-decreasing).  The call
 * admits each block at its arrival time (later, in arrival order, while
 * the server answers BUSY), dispatches, and returns when all are done;
 * latency_ns[i] = completion time - arrival time, samples_emitted[i] (may
 * be NULL) as for poll.  stats may be NULL (no statistics). */
int rfi_server_replay(rfi_server* srv, int64_t n_blocks, const uint32_t* stream_ids,
                      const int64_t* arrival_ns, const void* const* blocks, void* const* outs,
                      const int64_t* lengths, rfi_window_stats* const* stats,
                      int64_t* latency_ns, int64_t* samples_emitted);
int rfi_server_destroy(rfi_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* RFI_MAD_H */
