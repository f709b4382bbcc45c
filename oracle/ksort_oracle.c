/*
 * K-sort CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Literal implementation of arXiv 1107.3622, Section 1.1, Steps 1-6, for
 * double and float keys.  The body lives in ksort_oracle_impl.h and is
 * instantiated once per key type below.  Only the test suite, the package
 * smoke check and the benchmark's CPU-baseline leg may load this library.
 *
 * Pins: every function here is checked by the CPU test suite against facts
 * the paper or mathematics fixes (the Section 1.2 illustration, brute force
 * over all small permutations and multisets, the closed-form pivot index and
 * one-level arrangement, the exact mean comparison count of Quick sort, and
 * numpy's sort).
 */
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "ksort_oracle.h"

#define KEY_T double
#define SFX(name) name##_f64
#include "ksort_oracle_impl.h"
#undef KEY_T
#undef SFX

#define KEY_T float
#define SFX(name) name##_f32
#include "ksort_oracle_impl.h"
#undef KEY_T
#undef SFX
