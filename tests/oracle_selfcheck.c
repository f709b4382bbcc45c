/*
 * Memory-safety run of the CPU oracle, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py (host code
 * only).  Inputs come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
 * the same counter-based definition the Python generator module uses; each
 * result is compared with the C library's qsort.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "ksort_oracle.h"

static uint64_t sm64(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int cmp_d(const void *x, const void *y)
{
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

static int cmp_f(const void *x, const void *y)
{
    float a = *(const float *)x, b = *(const float *)y;
    return (a > b) - (a < b);
}

static int check_f64(int64_t n, uint64_t seed, int grid)
{
    double *a = malloc((size_t)(n ? n : 1) * sizeof(double));
    double *b = malloc((size_t)(n ? n : 1) * sizeof(double));
    for (int64_t t = 0; t < n; t++) {
        uint64_t z = sm64(seed, (uint64_t)t);
        a[t] = grid ? (double)(z >> 56) : (double)(z >> 11) * 0x1p-53;
    }
    memcpy(b, a, (size_t)n * sizeof(double));
    int64_t fp = 0, calls = 0, comps = 0;
    ksort_oracle_call tr[4];
    if (ksort_oracle_sort_f64(a, n, &fp, tr, 4, &calls, &comps) != 0)
        return 1;
    qsort(b, (size_t)n, sizeof(double), cmp_d);
    int bad = n ? memcmp(a, b, (size_t)n * sizeof(double)) != 0 : 0;
    free(a);
    free(b);
    return bad;
}

static int check_f32(int64_t n, uint64_t seed)
{
    float *a = malloc((size_t)(n ? n : 1) * sizeof(float));
    float *b = malloc((size_t)(n ? n : 1) * sizeof(float));
    for (int64_t t = 0; t < n; t++)
        a[t] = (float)((double)(sm64(seed, (uint64_t)t) >> 40) * 0x1p-24);
    memcpy(b, a, (size_t)n * sizeof(float));
    int64_t fp = 0;
    if (ksort_oracle_sort_f32(a, n, &fp, NULL, 0, NULL, NULL) != 0)
        return 1;
    qsort(b, (size_t)n, sizeof(float), cmp_f);
    int bad = n ? memcmp(a, b, (size_t)n * sizeof(float)) != 0 : 0;
    free(a);
    free(b);
    return bad;
}

int main(void)
{
    int bad = 0;
    for (int64_t n = 0; n <= 600; n++) {
        bad += check_f64(n, 1000 + (uint64_t)n, 0);
        bad += check_f64(n, 2000 + (uint64_t)n, 1);
        bad += check_f32(n, 3000 + (uint64_t)n);
    }
    bad += check_f64(100000, 1, 0);
    bad += check_f64(100000, 2, 1);
    bad += check_f32(100000, 3);
    /* partition_level and segmented on a small batch */
    double a[64];
    for (int t = 0; t < 64; t++)
        a[t] = (double)(sm64(9, (uint64_t)t) >> 58);
    int64_t left[3] = {0, 10, 63}, len[3] = {10, 53, 1}, piv[3];
    bad += ksort_oracle_partition_level_f64(a, left, len, 3, piv) != 0;
    int64_t offs[4] = {0, 5, 5, 64}, fps[3];
    bad += ksort_oracle_segmented_f64(a, offs, 3, fps) != 0;
    printf("selfcheck failures: %d\n", bad);
    return bad ? 1 : 0;
}
