"""GPU parity of the literal arrangement (Steps 1-4 exactly as the
sequential steps leave the array): one level on many segments equals the
oracle's in every position, and the whole sort makes exactly the oracle's
calls (segment and pivot index of every call) and ends with its array."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_bit_equal, note, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

ILLUSTRATION = [55, 66, 60, 78, 22, 50, 75, 5, 8, 94]  # Section 1.2


def random_segments(seed: int, n: int, maxlen: int, gaps: bool = True):
    lens = synth.loguniform_int(seed, n // 2 + 8, 1, maxlen)
    gap = synth.loguniform_int(seed + 1, lens.size, 1, 64) - 1 if gaps else np.zeros(lens.size, dtype=np.int64)
    left, lengths, pos = [], [], 0
    for g, L in zip(gap, lens):
        pos += int(g)
        if pos + int(L) > n:
            break
        left.append(pos)
        lengths.append(int(L))
        pos += int(L)
    return np.array(left, dtype=np.int64), np.array(lengths, dtype=np.int64)


def keys(kind: str, seed: int, n: int, dtype) -> np.ndarray:
    a = synth.uniform_f64(seed, n)
    if kind == "ties":
        a = np.floor(a * 8)
    elif kind == "sorted":
        a = np.sort(a)
    elif kind == "equal":
        a = np.full(n, 0.25)
    elif kind == "organ":
        a = np.concatenate([np.arange(n // 2), np.arange(n - n // 2)[::-1]]).astype(np.float64)
    return a.astype(dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,maxlen,kind", [(5000, 40, "ties"), (200_000, 5000, "uniform"),
                                           (1_000_000, 300_000, "uniform"), (50_000, 50_000, "ties")])
def test_level_exact_vs_oracle(dtype, n, maxlen, kind):
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    a = keys(kind, n + maxlen, n, dtype)
    left, length = random_segments(n, n, maxlen)
    note(f"level_exact n={n} nseg={left.size} kind={kind} dtype={np.dtype(dtype).name}")
    sentinel = -7.0
    d_out = torch.full((n,), sentinel, dtype=torch.float64 if dtype == np.float64 else torch.float32, device="cuda")
    piv = to_host(ksort.ksort_partition_level_exact(to_dev(a), d_out, to_dev(left), to_dev(length)))
    out = to_host(d_out)
    b = a.copy()
    want = oracle.partition_level_(b, left, length)
    assert np.array_equal(piv, want)
    covered = np.zeros(n, dtype=bool)
    for s in range(left.size):
        covered[left[s]:left[s] + length[s]] = True
    assert_bit_equal(out[covered], b[covered], "arrangement inside the segments")
    assert np.all(out[~covered] == sentinel)


def test_level_exact_whole_array_and_tiny_segments():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    for n in (1, 2, 3, 4095, 4096, 4097, 12289):
        for kind in ("uniform", "ties", "sorted", "equal", "organ"):
            a = keys(kind, n, n, np.float64)
            note(f"level_exact whole n={n} kind={kind}")
            d_out = torch.empty(n, dtype=torch.float64, device="cuda")
            piv = to_host(ksort.ksort_partition_level_exact(to_dev(a), d_out, to_dev(np.array([0], dtype=np.int64)),
                                                           to_dev(np.array([n], dtype=np.int64))))
            b = a.copy()
            i, _ = oracle.partition_(b, 0, n - 1)
            assert int(piv[0]) == i
            assert_bit_equal(to_host(d_out), b, f"whole-array call n={n} {kind}")
    # every segment of one and two keys
    a = keys("ties", 3, 1000, np.float64)
    left = np.arange(0, 1000, 3, dtype=np.int64)[:-1]
    length = np.where(np.arange(left.size) % 2 == 0, 1, 2).astype(np.int64)
    d_out = torch.zeros(1000, dtype=torch.float64, device="cuda")
    piv = to_host(ksort.ksort_partition_level_exact(to_dev(a), d_out, to_dev(left), to_dev(length)))
    b = a.copy()
    assert np.array_equal(piv, oracle.partition_level_(b, left, length))
    out = to_host(d_out)
    for s in range(left.size):
        assert_bit_equal(out[left[s]:left[s] + length[s]], b[left[s]:left[s] + length[s]], "short segments")


def test_level_exact_rejects_bad_segments():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    d_in = torch.arange(100, dtype=torch.float64, device="cuda").flip(0).contiguous()
    d_out = torch.zeros_like(d_in)
    for left, length in (([0, 5], [10, 10]), ([0, 95], [10, 10]), ([-1], [5]), ([3], [0])):
        note(f"bad exact segments {left} {length}")
        with pytest.raises(ksort.KsortError):
            ksort.ksort_partition_level_exact(d_in, d_out, to_dev(np.array(left, dtype=np.int64)),
                                              to_dev(np.array(length, dtype=np.int64)))


def oracle_calls(a: np.ndarray):
    b = a.copy()
    info = oracle.sort_(b, trace_cap=0)
    full = oracle.sort_(a.copy(), trace_cap=info["calls"])
    calls = np.array([(t["left"], t["right"], t["i"]) for t in full["trace"]], dtype=np.int64).reshape(-1, 3)
    return b, info["first_pivot"], calls


def sorted_rows(c: np.ndarray) -> np.ndarray:
    c = np.asarray(c).reshape(-1, 3)
    return c[np.lexsort((c[:, 2], c[:, 1], c[:, 0]))]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,kind", [(1, "uniform"), (2, "uniform"), (3, "ties"), (1000, "uniform"),
                                    (20_000, "ties"), (100_000, "uniform"), (3000, "sorted"),
                                    (2000, "equal"), (4001, "organ")])
def test_sort_exact_makes_the_oracle_calls(dtype, n, kind):
    from paper_1107_3622_amd import ksort
    a = keys(kind, 11 + n, n, dtype)
    want, wfp, wcalls = oracle_calls(a)
    note(f"sort_exact n={n} kind={kind} dtype={np.dtype(dtype).name} calls={len(wcalls)}")
    t = to_dev(a)
    fp, ncalls, calls = ksort.ksort_sort_exact(t, calls_cap=max(len(wcalls), 1))
    assert fp == wfp
    assert ncalls == len(wcalls)
    assert_bit_equal(to_host(t), want, "sorted array")
    if ncalls:
        assert np.array_equal(sorted_rows(to_host(calls)), sorted_rows(wcalls))


def test_sort_exact_illustration():
    from paper_1107_3622_amd import ksort
    a = np.array(ILLUSTRATION, dtype=np.float64)
    want, wfp, wcalls = oracle_calls(a)
    note("sort_exact illustration")
    t = to_dev(a)
    fp, ncalls, calls = ksort.ksort_sort_exact(t, calls_cap=16)
    assert fp == 4 == wfp
    assert to_host(t).tolist() == sorted(ILLUSTRATION)
    # the six calls of the trace: [0,9] i=4, [0,3], [2,3], [5,9], [7,9], [8,9]
    assert np.array_equal(sorted_rows(to_host(calls)), sorted_rows(wcalls))
    assert [tuple(r[:2]) for r in sorted_rows(wcalls)] == [(0, 3), (0, 9), (2, 3), (5, 9), (7, 9), (8, 9)]


def test_sort_exact_full_size_and_call_count():
    from paper_1107_3622_amd import ksort
    n = 7_000_000
    a = synth.uniform_f64(4, n)
    b = a.copy()
    info = oracle.sort_(b)
    note(f"sort_exact n={n}")
    t = to_dev(a)
    fp, ncalls, _ = ksort.ksort_sort_exact(t)
    assert fp == info["first_pivot"]
    assert ncalls == info["calls"]
    assert_bit_equal(to_host(t), b, "sorted array at 7e6")


def test_sort_exact_rejects_bad_arguments():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    lib = ksort.load()
    t = torch.zeros(10, dtype=torch.float64, device="cuda")
    assert lib.ksort_sort_exact(9, t.data_ptr(), 10, None, None, 0, None, None) == -1
    assert lib.ksort_sort_exact(0, t.data_ptr(), -1, None, None, 0, None, None) == -1
    assert lib.ksort_sort_exact(0, None, 10, None, None, 0, None, None) == -1
    assert lib.ksort_sort_exact(0, t.data_ptr(), 10, None, t.data_ptr(), 1, None, None) == -1
