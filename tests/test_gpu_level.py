"""GPU parity of one partition level (Steps 1-4) on many segments:
pivot index equal to the oracle's, each side the same multiset as the
oracle's, the partition property, and nothing outside the segments
written."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import note, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


def random_segments(rng_seed: int, n: int, maxlen: int):
    lens = synth.loguniform_int(rng_seed, n // 2 + 8, 1, maxlen)
    gaps = synth.loguniform_int(rng_seed + 1, lens.size, 1, 64) - 1
    left, lengths, pos = [], [], 0
    for g, L in zip(gaps, lens):
        pos += int(g)
        if pos + int(L) > n:
            break
        left.append(pos)
        lengths.append(int(L))
        pos += int(L)
    return np.array(left, dtype=np.int64), np.array(lengths, dtype=np.int64)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,maxlen", [(5000, 40), (200_000, 5000), (1_000_000, 300_000)])
def test_partition_level_vs_oracle(dtype, n, maxlen):
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    a = synth.uniform_f64(n + maxlen, n).astype(dtype)
    if maxlen == 40:
        a = np.floor(a * 8).astype(dtype)  # many ties with the key
    left, length = random_segments(n, n, maxlen)
    note(f"partition_level n={n} nseg={left.size} dtype={np.dtype(dtype).name}")
    d_in = to_dev(a)
    sentinel = -7.0
    d_out = torch.full_like(d_in, sentinel)
    piv = to_host(ksort.ksort_partition_level(d_in, d_out, to_dev(left), to_dev(length)))
    out = to_host(d_out)
    b = a.copy()
    want = oracle.partition_level_(b, left, length)
    assert np.array_equal(piv, want)
    covered = np.zeros(n, dtype=bool)
    for s in range(left.size):
        lo, hi, i = int(left[s]), int(left[s] + length[s]), int(piv[s])
        covered[lo:hi] = True
        key = a[lo]
        assert out[i] == key
        assert np.all(out[lo:i] < key) and np.all(key <= out[i + 1:hi])
        assert np.array_equal(np.sort(out[lo:i]), np.sort(b[lo:i]))
        assert np.array_equal(np.sort(out[i + 1:hi]), np.sort(b[i + 1:hi]))
    assert np.all(out[~covered] == sentinel)


def test_partition_level_rejects_bad_segments():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    d_in = torch.arange(100, dtype=torch.float64, device="cuda").flip(0).contiguous()
    d_out = torch.zeros_like(d_in)
    for left, length in (([0, 95], [10, 10]), ([-1], [5]), ([3], [0])):
        note(f"bad segments {left} {length}")
        with pytest.raises(ksort.KsortError):
            ksort.ksort_partition_level(d_in, d_out, to_dev(np.array(left, dtype=np.int64)),
                                        to_dev(np.array(length, dtype=np.int64)))
