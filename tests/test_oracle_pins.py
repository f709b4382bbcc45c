"""CPU oracle pinned to the paper and to mathematics (no GPU needed).

Each test runs one pin from tests/pins.py at full size; the mutation tests
run the same pins against broken copies of the oracle.
"""
import numpy as np
import pytest

import oracle
import pins


def test_illustration(oracle_lib):
    assert pins.check_illustration(oracle_lib) == []


def test_all_permutations_up_to_8(oracle_lib):
    assert pins.check_permutations(oracle_lib, nmax=8) == []


def test_all_small_multisets(oracle_lib):
    # {0,1,2}^n for n <= 9 and {0,1,2,3}^n for n <= 7: keys equal to the key
    # must go right, and runs of equal keys must still terminate.
    assert pins.check_multisets(oracle_lib, spec=((3, 9), (4, 7))) == []


def test_mean_comparisons_equal_knuth_exactly(oracle_lib):
    assert pins.check_mean_comparisons(oracle_lib, nmax=8) == []


def test_knuth_formula_values():
    # 2(n+1)H_n - 4n: n = 10 gives 24.4373..., n = 8 gives 2369/140.
    from fractions import Fraction
    assert pins.knuth_mean_comparisons(8) == Fraction(2369, 140)
    assert abs(float(pins.knuth_mean_comparisons(10)) - 24.437301587) < 1e-8


def test_library_sort_bit_exact(oracle_lib):
    assert pins.check_library_sort(oracle_lib) == []


def test_levels_and_batches(oracle_lib):
    assert pins.check_levels_and_batches(oracle_lib) == []


def test_edge_cases(oracle_lib):
    for n in (0, 1):
        a = np.zeros(n)
        info = oracle.sort_(a, lib=oracle_lib)
        assert info["calls"] == 0
        assert info["first_pivot"] == (-1 if n == 0 else 0)
    # all-equal: every key goes right, depth n - 1, still sorted
    a = np.full(300, 0.5)
    info = oracle.sort_(a, lib=oracle_lib)
    assert info["calls"] == 299 and info["first_pivot"] == 0
    # sorted and reverse-sorted: the quadratic case of Section 5
    a = np.arange(500, dtype=np.float64)
    info = oracle.sort_(a, lib=oracle_lib)
    assert info["comparisons"] == 499 * 500 // 2
    assert np.array_equal(a, np.arange(500.0))
    a = np.arange(500, dtype=np.float64)[::-1].copy()
    oracle.sort_(a, lib=oracle_lib)
    assert np.array_equal(a, np.arange(500.0))


def test_f32_uses_f32_comparisons(oracle_lib):
    # Two doubles that round to the same float must compare equal in the
    # f32 oracle (they are the same float key).
    a = np.array([1.0, 1.0 + 2**-30, 0.5], dtype=np.float64).astype(np.float32)
    assert a[0] == a[1]
    i, rec = oracle.partition_(a, 0, 2, lib=oracle_lib)
    assert i == 1 and rec["temp"] == 1.0


def test_nan_goes_left(oracle_lib):
    # key <= NaN is false, so the NaN is placed left of the key.
    a = np.array([0.5, np.nan, 0.7, 0.1])
    i, _ = oracle.partition_(a, 0, 3, lib=oracle_lib)
    assert i == 2 and np.isnan(a[:2]).sum() == 1


@pytest.mark.parametrize("threads", [2, 5, 8])
def test_parallel_driver_equals_one_thread(oracle_lib, threads):
    # The task-parallel driver runs the same literal calls on sub-arrays that
    # share no element; its array and first pivot must equal the one-thread
    # run's (and numpy's order), bit for bit, including tie-heavy and
    # ordered inputs and sizes around the task grain.
    import synth
    cases = [synth.uniform_f64(21, 700_000), np.floor(synth.uniform_f64(22, 300_000) * 16),
             np.sort(synth.uniform_f64(23, 6000)), synth.uniform_f64(24, 4096),
             synth.uniform_f64(25, 4097), synth.uniform_f64(26, 2), np.zeros(0),
             synth.uniform_f64(27, 500_000).astype(np.float32)]
    for a in cases:
        b = a.copy()
        info = oracle.sort_(b, lib=oracle_lib)
        c = a.copy()
        fp = oracle.sort_parallel_(c, threads, lib=oracle_lib)
        assert np.array_equal(b.view(np.uint8), c.view(np.uint8))
        assert np.array_equal(c, np.sort(a))
        assert fp == info["first_pivot"]
