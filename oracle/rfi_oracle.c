/*
 * rfi_oracle.c -- plain, slow, obviously-correct CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the product path.  It
 * shares no code with the GPU library.  Every window is handled by the
 * textbook definition: a full sort for the median, a full sort of the
 * absolute deviations for the MAD, one binary32 formula for the threshold
 * and a per-sample comparison and replacement.
 *
 * Paper: Buch et al., "Implementing and Characterizing Real-time Broadband
 * RFI Excision for the GMRT Wideband Backend", Sec. II-D, Eqs. (1)-(2).
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread (binary32 floats
 * on SSE, no fused multiply-add).
 */
#include "rfi_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x64-10, from the description in Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds;  */
/* each round multiplies counter words 0 and 2 by two fixed odd        */
/* multipliers, and builds the new counter from the high halves xored  */
/* with the other words and the round key, and the low halves; the key */
/* advances by two Weyl increments between rounds.                     */
/* ------------------------------------------------------------------ */
static const uint64_t PHILOX_MUL0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_MUL1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_WEYL0 = 0x9E3779B97F4A7C15ULL; /* golden ratio  */
static const uint64_t PHILOX_WEYL1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1   */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL0;
            k1 += PHILOX_WEYL1;
        }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_MUL0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_MUL1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------ */
/* Q8 Gaussian quantile table for the digital-noise replacement.       */
/* The standard normal quantile is found by bisection on               */
/* Phi(z) = erfc(-z / sqrt 2) / 2 until the bracket stops shrinking.   */
/* ------------------------------------------------------------------ */
static double std_normal_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

static double std_normal_quantile(double p)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (std_normal_cdf(mid) < p) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static int16_t g_q8[4096];
static pthread_once_t g_q8_once = PTHREAD_ONCE_INIT;

static void q8_init(void)
{
    for (int u = 0; u < 4096; ++u) {
        double z = std_normal_quantile((u + 0.5) / 4096.0);
        g_q8[u] = (int16_t)lround(256.0 * z);
    }
}

void orc_q8_table(int16_t out[4096])
{
    pthread_once(&g_q8_once, q8_init);
    memcpy(out, g_q8, sizeof(g_q8));
}

/* ------------------------------------------------------------------ */
/* Layout                                                              */
/* ------------------------------------------------------------------ */
int64_t orc_layout(int32_t n_streams, const int64_t* lengths, const int32_t* windows,
                   int64_t* sample_offsets, int64_t* window_offsets)
{
    int64_t samples = 0, wins = 0;
    for (int32_t s = 0; s < n_streams; ++s) {
        if (lengths[s] < 0 || windows[s] < 1) return -1;
        if (sample_offsets) sample_offsets[s] = samples;
        if (window_offsets) window_offsets[s] = wins;
        samples += ((lengths[s] + 63) / 64) * 64;
        wins += (lengths[s] + windows[s] - 1) / windows[s];
    }
    return wins;
}

/* ------------------------------------------------------------------ */
/* One window, by definition.                                          */
/* ------------------------------------------------------------------ */
static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static int32_t saturate(int64_t v, int32_t vmin, int32_t vmax)
{
    if (v < vmin) return vmin;
    if (v > vmax) return vmax;
    return (int32_t)v;
}

/* floor(a / 65536) for any sign of a: the rounding of the Q8 x Q8 product. */
static int64_t floor_div_65536(int64_t a)
{
    int64_t q = a / 65536;
    if (a % 65536 != 0 && a < 0) q -= 1;
    return q;
}

/* Noise offset q(j) for absolute sample index j of stream `stream`.
 * One Philox4x64-10 block (key (seed, stream), counter (j >> 2, 0, 0, 0))
 * serves 4 consecutive samples: sample j takes word j & 3 of the block and
 * uses its 12 most significant bits as the table index. */
static int64_t noise_offset(int64_t j, uint32_t stream, uint64_t seed, int32_t sigma_q8)
{
    uint64_t ctr[4] = {(uint64_t)j >> 2, 0, 0, 0};
    uint64_t key[2] = {seed, (uint64_t)stream};
    uint64_t r[4];
    orc_philox4x64_10(ctr, key, r);
    uint64_t word = r[j & 3];
    uint32_t u = (uint32_t)(word >> 52);
    pthread_once(&g_q8_once, q8_init);
    return floor_div_65536((int64_t)sigma_q8 * (int64_t)g_q8[u] + 32768);
}

static void window_apply(const int32_t* X, int32_t* Y, int32_t n, int32_t m, int32_t D,
                         int32_t D_thr, int64_t abs_start, uint32_t stream, uint64_t seed,
                         float k, int32_t mode, int32_t vmin, int32_t vmax, orc_stats* st);

/* X, Y: n samples widened to int32; vmin/vmax: the dtype's range. */
static void window_core(const int32_t* X, int32_t* Y, int32_t n, int64_t abs_start,
                        uint32_t stream, uint64_t seed, float k, int32_t mode,
                        int32_t vmin, int32_t vmax, orc_stats* st)
{
    int32_t* s = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t r = (n - 1) / 2;

    /* Median: sort the window, take rank r (lower median for even n). */
    memcpy(s, X, (size_t)n * sizeof(int32_t));
    qsort(s, (size_t)n, sizeof(int32_t), cmp_i32);
    int32_t m = s[r];

    /* MAD: sort |x - m|, take the same rank. */
    for (int32_t i = 0; i < n; ++i) s[i] = abs(X[i] - m);
    qsort(s, (size_t)n, sizeof(int32_t), cmp_i32);
    int32_t D = s[r];
    free(s);
    window_apply(X, Y, n, m, D, D, abs_start, stream, seed, k, mode, vmin, vmax, st);
}

/* Eq. (1)-(2) for one window whose median m and MAD D are known, with the
 * threshold taken from D_thr (D itself, or the median of MADs of Eq. (3)). */
static void window_apply(const int32_t* X, int32_t* Y, int32_t n, int32_t m, int32_t D,
                         int32_t D_thr, int64_t abs_start, uint32_t stream, uint64_t seed,
                         float k, int32_t mode, int32_t vmin, int32_t vmax, orc_stats* st)
{
    /* Eq. (1): robust sigma 1.4826 * D, threshold n_sigma times it. */
    float sigma = 1.4826f * (float)D_thr;
    float t = k * sigma;
    int32_t T = (int32_t)floorf(t);
    int32_t sigma_q8 = (int32_t)(sigma * 256.0f);

    /* Eq. (2): replace samples outside the thresholds. */
    uint32_t flagged = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t dev = X[i] - m;
        int32_t d = abs(dev);
        if ((float)d > t) {
            ++flagged;
            if (mode == ORC_ZERO) {
                Y[i] = 0;
            } else if (mode == ORC_CLIP) {
                int32_t sgn = dev > 0 ? 1 : -1;
                Y[i] = saturate((int64_t)m + (int64_t)sgn * T, vmin, vmax);
            } else {
                int64_t q = noise_offset(abs_start + i, stream, seed, sigma_q8);
                Y[i] = saturate((int64_t)m + q, vmin, vmax);
            }
        } else {
            Y[i] = X[i];
        }
    }
    if (st) {
        st->median = m;
        st->mad = D;
        st->n_flagged = flagged;
        st->threshold = t;
    }
}

void orc_window_i8(const int8_t* x, int8_t* y, int32_t n, int64_t abs_start,
                   uint32_t stream, uint64_t seed, float k, int32_t mode, orc_stats* st)
{
    if (n < 1) return;
    int32_t* X = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* Y = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) X[i] = x[i];
    window_core(X, Y, n, abs_start, stream, seed, k, mode, -128, 127, st);
    for (int32_t i = 0; i < n; ++i) y[i] = (int8_t)Y[i];
    free(X);
    free(Y);
}

void orc_window_i16(const int16_t* x, int16_t* y, int32_t n, int64_t abs_start,
                    uint32_t stream, uint64_t seed, float k, int32_t mode, orc_stats* st)
{
    if (n < 1) return;
    int32_t* X = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* Y = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) X[i] = x[i];
    window_core(X, Y, n, abs_start, stream, seed, k, mode, -32768, 32767, st);
    for (int32_t i = 0; i < n; ++i) y[i] = (int16_t)Y[i];
    free(X);
    free(Y);
}

/* ------------------------------------------------------------------ */
/* Whole batch: a flat list of (stream, window) items split evenly     */
/* over POSIX threads.                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int elem_size;
    const void* x;
    void* y;
    int32_t n_streams;
    const int64_t* lengths;
    const int32_t* windows;
    const float* k;
    const int32_t* mode;
    uint64_t seed;
    orc_stats* stats;
    const int64_t* soff;
    const int64_t* woff;
    int64_t first, last; /* window items [first, last) */
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* j = (batch_job*)arg;
    int32_t s = 0;
    for (int64_t item = j->first; item < j->last; ++item) {
        while (s + 1 < j->n_streams && j->woff[s + 1] <= item) ++s;
        while (j->woff[s] > item) --s;
        int64_t w = item - j->woff[s];
        int64_t a = w * j->windows[s];
        int64_t rem = j->lengths[s] - a;
        int32_t n = (int32_t)(rem < j->windows[s] ? rem : j->windows[s]);
        orc_stats* st = j->stats ? &j->stats[item] : NULL;
        if (j->elem_size == 1) {
            const int8_t* xs = (const int8_t*)j->x + j->soff[s] + a;
            int8_t* ys = (int8_t*)j->y + j->soff[s] + a;
            orc_window_i8(xs, ys, n, a, (uint32_t)s, j->seed, j->k[s], j->mode[s], st);
        } else {
            const int16_t* xs = (const int16_t*)j->x + j->soff[s] + a;
            int16_t* ys = (int16_t*)j->y + j->soff[s] + a;
            orc_window_i16(xs, ys, n, a, (uint32_t)s, j->seed, j->k[s], j->mode[s], st);
        }
    }
    return NULL;
}

static int filter_batch(int elem_size, const void* x, void* y, int32_t n_streams,
                        const int64_t* lengths, const int32_t* windows, const float* k,
                        const int32_t* mode, uint64_t seed, orc_stats* stats, int32_t n_threads)
{
    if (n_streams < 0) return -1;
    if (n_streams == 0) return 0;
    int64_t* soff = (int64_t*)malloc((size_t)n_streams * sizeof(int64_t));
    int64_t* woff = (int64_t*)malloc((size_t)n_streams * sizeof(int64_t));
    int64_t total = orc_layout(n_streams, lengths, windows, soff, woff);
    for (int32_t s = 0; s < n_streams && total >= 0; ++s)
        if (mode[s] < ORC_ZERO || mode[s] > ORC_NOISE || !(k[s] >= 0.0f)) total = -1;
    if (total < 0) {
        free(soff);
        free(woff);
        return -1;
    }
    pthread_once(&g_q8_once, q8_init); /* build the table before threads start */
    if (n_threads < 1) n_threads = 1;
    if (n_threads > total && total > 0) n_threads = (int32_t)total;
    pthread_t* tid = (pthread_t*)malloc((size_t)n_threads * sizeof(pthread_t));
    batch_job* jobs = (batch_job*)malloc((size_t)n_threads * sizeof(batch_job));
    for (int32_t i = 0; i < n_threads; ++i) {
        batch_job j = {elem_size, x, y, n_streams, lengths, windows, k, mode, seed, stats,
                       soff, woff, total * i / n_threads, total * (i + 1) / n_threads};
        jobs[i] = j;
        pthread_create(&tid[i], NULL, batch_worker, &jobs[i]);
    }
    for (int32_t i = 0; i < n_threads; ++i) pthread_join(tid[i], NULL);
    free(tid);
    free(jobs);
    free(soff);
    free(woff);
    return 0;
}

int orc_filter_i8(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                  const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                  orc_stats* stats, int32_t n_threads)
{
    return filter_batch(1, x, y, n_streams, lengths, windows, k, mode, seed, stats, n_threads);
}

int orc_filter_i16(const int16_t* x, int16_t* y, int32_t n_streams, const int64_t* lengths,
                   const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                   orc_stats* stats, int32_t n_threads)
{
    return filter_batch(2, x, y, n_streams, lengths, windows, k, mode, seed, stats, n_threads);
}

/* ------------------------------------------------------------------ */
/* Median of MADs (Eq. (3)).                                           */
/* ------------------------------------------------------------------ */
/* Lower median and MAD of n int8 samples (the definitions of window_core). */
static void median_mad(const int32_t* X, int32_t n, int32_t* m_out, int32_t* D_out)
{
    int32_t* s = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t r = (n - 1) / 2;
    memcpy(s, X, (size_t)n * sizeof(int32_t));
    qsort(s, (size_t)n, sizeof(int32_t), cmp_i32);
    int32_t m = s[r];
    for (int32_t i = 0; i < n; ++i) s[i] = abs(X[i] - m);
    qsort(s, (size_t)n, sizeof(int32_t), cmp_i32);
    *m_out = m;
    *D_out = s[r];
    free(s);
}

typedef struct {
    const int8_t* x;
    int8_t* y;
    int32_t n_streams;
    const int64_t* lengths;
    const int32_t* windows;
    const float* k;
    const int32_t* mode;
    int32_t mom_k;
    uint64_t seed;
    orc_stats* stats;
    const int64_t* soff;
    const int64_t* woff;
    int32_t first, last; /* streams [first, last) */
} mom_job;

/* One stream: M(x) and D of every window; M_m(w) = lower median of the MADs
 * of the K windows ending at w (fewer at the stream's start); then Eqs.
 * (1)-(2) with M_m(w) in place of the window's own D. */
static void mom_stream(const mom_job* j, int32_t s)
{
    const int64_t L = j->lengths[s];
    const int32_t W = j->windows[s];
    const int64_t nw = (L + W - 1) / W;
    if (nw == 0) return;
    int32_t* med = (int32_t*)malloc((size_t)nw * sizeof(int32_t));
    int32_t* mad = (int32_t*)malloc((size_t)nw * sizeof(int32_t));
    int32_t* X = (int32_t*)malloc((size_t)W * sizeof(int32_t));
    int32_t* Y = (int32_t*)malloc((size_t)W * sizeof(int32_t));
    int32_t* sorted = (int32_t*)malloc((size_t)j->mom_k * sizeof(int32_t));
    const int8_t* xs = j->x + j->soff[s];
    int8_t* ys = j->y + j->soff[s];
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t a = w * W;
        const int32_t n = (int32_t)(L - a < W ? L - a : W);
        for (int32_t i = 0; i < n; ++i) X[i] = xs[a + i];
        median_mad(X, n, &med[w], &mad[w]);
    }
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t lo = w + 1 > j->mom_k ? w + 1 - j->mom_k : 0;
        const int32_t cnt = (int32_t)(w + 1 - lo);
        memcpy(sorted, mad + lo, (size_t)cnt * sizeof(int32_t));
        qsort(sorted, (size_t)cnt, sizeof(int32_t), cmp_i32);
        const int32_t Dm = sorted[(cnt - 1) / 2];
        const int64_t a = w * W;
        const int32_t n = (int32_t)(L - a < W ? L - a : W);
        for (int32_t i = 0; i < n; ++i) X[i] = xs[a + i];
        orc_stats* st = j->stats ? &j->stats[j->woff[s] + w] : NULL;
        window_apply(X, Y, n, med[w], mad[w], Dm, a, (uint32_t)s, j->seed, j->k[s], j->mode[s],
                     -128, 127, st);
        for (int32_t i = 0; i < n; ++i) ys[a + i] = (int8_t)Y[i];
    }
    free(med);
    free(mad);
    free(X);
    free(Y);
    free(sorted);
}

static void* mom_worker(void* arg)
{
    const mom_job* j = (const mom_job*)arg;
    for (int32_t s = j->first; s < j->last; ++s) mom_stream(j, s);
    return NULL;
}

int orc_mom_filter_i8(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                      const int32_t* windows, const float* k, const int32_t* mode, int32_t mom_k,
                      uint64_t seed, orc_stats* stats, int32_t n_threads)
{
    if (n_streams < 0 || mom_k < 1) return -1;
    if (n_streams == 0) return 0;
    int64_t* soff = (int64_t*)malloc((size_t)n_streams * sizeof(int64_t));
    int64_t* woff = (int64_t*)malloc((size_t)n_streams * sizeof(int64_t));
    int64_t total = orc_layout(n_streams, lengths, windows, soff, woff);
    for (int32_t s = 0; s < n_streams && total >= 0; ++s)
        if (mode[s] < ORC_ZERO || mode[s] > ORC_NOISE || !(k[s] >= 0.0f)) total = -1;
    if (total < 0) {
        free(soff);
        free(woff);
        return -1;
    }
    pthread_once(&g_q8_once, q8_init);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_streams) n_threads = n_streams;
    pthread_t* tid = (pthread_t*)malloc((size_t)n_threads * sizeof(pthread_t));
    mom_job* jobs = (mom_job*)malloc((size_t)n_threads * sizeof(mom_job));
    for (int32_t i = 0; i < n_threads; ++i) {
        mom_job j = {x, y, n_streams, lengths, windows, k, mode, mom_k, seed, stats, soff, woff,
                     (int32_t)((int64_t)n_streams * i / n_threads),
                     (int32_t)((int64_t)n_streams * (i + 1) / n_threads)};
        jobs[i] = j;
        pthread_create(&tid[i], NULL, mom_worker, &jobs[i]);
    }
    for (int32_t i = 0; i < n_threads; ++i) pthread_join(tid[i], NULL);
    free(tid);
    free(jobs);
    free(soff);
    free(woff);
    return 0;
}
