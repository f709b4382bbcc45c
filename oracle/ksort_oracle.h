/*
 * K-sort CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, literal C implementation of K-sort (Sundararajan, Pal,
 * Chakraborty, Mahanti, arXiv 1107.3622, Section 1.1, Steps 1-6).  It exists
 * only to check the HIP library: only the test suite, the package smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or table with the HIP library and includes nothing from it.
 *
 * Key types: double (suffix _f64) and float (suffix _f32).  The paper does
 * not state its key type (Section 2 only says U[0,1] variates); both widths
 * are provided and compare in their own precision.
 *
 * Readings of the text (where it is silent or garbled) are listed in the
 * implementation file next to the step they affect.
 */
#ifndef KSORT_ORACLE_H
#define KSORT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One partition call (Steps 1-4) as the literal algorithm performed it. */
typedef struct ksort_oracle_call {
    int64_t left;         /* segment [left, right] */
    int64_t right;
    int64_t i;            /* final index of the key (Step-4) */
    int64_t comparisons;  /* executions of the Step-3 comparison */
    int64_t k_minus_i;    /* k - i at loop exit (the text's k tracks i + 1) */
    double key;           /* a[left] at entry */
    double temp;          /* Step-3.1 temp; meaningful only when flag == 1 */
    int32_t flag;         /* Step-3.1 flag at Step-4 */
    int32_t pad;
} ksort_oracle_call;

/* Steps 1-4 on a[left..right] (right >= left).  Returns the key's final
 * index i.  `rec` may be NULL. */
int64_t ksort_oracle_partition_f64(double *a, int64_t left, int64_t right,
                                   ksort_oracle_call *rec);
int64_t ksort_oracle_partition_f32(float *a, int64_t left, int64_t right,
                                   ksort_oracle_call *rec);

/* Steps 1-6 on a[0..n-1], in place, depth-first and left side first.
 *   first_pivot : (nullable) receives i of the first partition call, 0 when
 *                 n == 1 and -1 when n == 0.
 *   trace       : (nullable) receives up to trace_cap call records in call
 *                 order; *ncalls (nullable) receives the total number of
 *                 calls, *ncomparisons (nullable) the total comparisons.
 * Returns 0, or -2 when the explicit stack cannot be allocated. */
int ksort_oracle_sort_f64(double *a, int64_t n, int64_t *first_pivot,
                          ksort_oracle_call *trace, int64_t trace_cap,
                          int64_t *ncalls, int64_t *ncomparisons);
int ksort_oracle_sort_f32(float *a, int64_t n, int64_t *first_pivot,
                          ksort_oracle_call *trace, int64_t trace_cap,
                          int64_t *ncalls, int64_t *ncomparisons);

/* Steps 1-6 on a[0..n-1] with up to `threads` threads: the top of the
 * recursion on the calling thread, then whole independent sub-arrays on the
 * threads, each call the literal one.  The final array equals
 * ksort_oracle_sort's; first_pivot as there.  Returns 0 or -2. */
int ksort_oracle_sort_parallel_f64(double *a, int64_t n, int threads, int64_t *first_pivot);
int ksort_oracle_sort_parallel_f32(float *a, int64_t n, int threads, int64_t *first_pivot);

/* One partition call (Steps 1-4) on each segment [left[s], left[s]+len[s]-1]
 * (len[s] >= 1, segments disjoint); pivot[s] receives i.  Returns 0, or -1
 * on a segment with len < 1. */
int ksort_oracle_partition_level_f64(double *a, const int64_t *left,
                                     const int64_t *len, int64_t nseg,
                                     int64_t *pivot);
int ksort_oracle_partition_level_f32(float *a, const int64_t *left,
                                     const int64_t *len, int64_t nseg,
                                     int64_t *pivot);

/* Steps 1-6 on each array [offsets[s], offsets[s+1]) independently;
 * first_pivots[s] (nullable) receives the first call's i relative to
 * offsets[s] (0 for a one-element array, -1 for an empty one). */
int ksort_oracle_segmented_f64(double *a, const int64_t *offsets, int64_t nseg,
                               int64_t *first_pivots);
int ksort_oracle_segmented_f32(float *a, const int64_t *offsets, int64_t nseg,
                               int64_t *first_pivots);

#ifdef __cplusplus
}
#endif

#endif /* KSORT_ORACLE_H */
