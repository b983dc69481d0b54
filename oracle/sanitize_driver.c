/* sanitize_driver.c -- TEST INFRASTRUCTURE: drives the oracle's C functions
 * over edge-case batches (empty streams, one-sample windows, short final
 * windows, saturated values, every mode, several threads) so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer can check its memory
 * accesses and arithmetic.  Prints "ok" and returns 0 when every call
 * succeeds; the sanitizers abort on their own findings. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "rfi_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 11);
}

static int run_i8(int n, const int64_t* L, const int32_t* W, int mode, int mom_k)
{
    int64_t* so = malloc(sizeof(int64_t) * (size_t)n);
    int64_t* wo = malloc(sizeof(int64_t) * (size_t)n);
    const int64_t nw = orc_layout(n, L, W, so, wo);
    int64_t total = 0;
    for (int s = 0; s < n; ++s) total += (L[s] + 63) / 64 * 64;
    int8_t* x = malloc((size_t)total + 1);
    int8_t* y = malloc((size_t)total + 1);
    orc_stats* st = malloc(sizeof(orc_stats) * (size_t)(nw + 1));
    float* k = malloc(sizeof(float) * (size_t)n);
    int32_t* m = malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < total; ++i) x[i] = (int8_t)(next_u32() % 7 == 0 ? (next_u32() & 1 ? 127 : -128)
                                                                             : (int)(next_u32() % 41) - 20);
    for (int s = 0; s < n; ++s) {
        k[s] = (float)(s % 4) * 1.5f;
        m[s] = mode;
    }
    int rc = mom_k > 0 ? orc_mom_filter_i8(x, y, n, L, W, k, m, mom_k, 7, st, 3)
                       : orc_filter_i8(x, y, n, L, W, k, m, 7, st, 3);
    free(so); free(wo); free(x); free(y); free(st); free(k); free(m);
    return rc;
}

static int run_i16(int n, const int64_t* L, const int32_t* W, int mode)
{
    int64_t total = 0;
    for (int s = 0; s < n; ++s) total += (L[s] + 63) / 64 * 64;
    const int64_t nw = orc_layout(n, L, W, NULL, NULL);
    int16_t* x = malloc(sizeof(int16_t) * (size_t)(total + 1));
    int16_t* y = malloc(sizeof(int16_t) * (size_t)(total + 1));
    orc_stats* st = malloc(sizeof(orc_stats) * (size_t)(nw + 1));
    float k[8];
    int32_t m[8];
    for (int64_t i = 0; i < total; ++i) x[i] = (int16_t)(next_u32() % 5 == 0 ? (next_u32() & 1 ? 32767 : -32768)
                                                                               : (int)(next_u32() % 2001) - 1000);
    for (int s = 0; s < n; ++s) {
        k[s] = 3.0f;
        m[s] = mode;
    }
    int rc = orc_filter_i16(x, y, n, L, W, k, m, 9, st, 2);
    free(x); free(y); free(st);
    return rc;
}

int main(void)
{
    const int64_t L[6] = {0, 1, 63, 4097, 700, 12345};
    const int32_t W[6] = {5, 1, 64, 4096, 7, 1000};
    for (int mode = 0; mode <= 2; ++mode) {
        if (run_i8(6, L, W, mode, 0) != 0) return 1;
        if (run_i16(6, L, W, mode) != 0) return 1;
        for (int K = 1; K <= 9; K += 4)
            if (run_i8(6, L, W, mode, K) != 0) return 1;
    }
    /* invalid arguments are rejected, not read past */
    const int64_t bad_L[1] = {-1};
    const int32_t one[1] = {4};
    if (orc_layout(1, bad_L, one, NULL, NULL) >= 0) return 1;
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x64_10(ctr, key, out);
    int16_t tab[4096];
    orc_q8_table(tab);
    printf("ok\n");
    return 0;
}
