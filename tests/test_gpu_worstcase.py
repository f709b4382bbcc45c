"""K-sort's worst cases on the GPU (the paper's average-case analysis,
Sections 1 and 4, assumes i.i.d. keys; ordered inputs and heavy duplicates
make every partition peel off a single key): sorted, reverse-sorted,
all-equal and few-distinct inputs sort bit-exactly as the oracle sorts
them, and the number of level passes is the depth that Steps 1-6 imply."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_bit_equal, note, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

N = 20_000
CUTOFF = 2048


def inputs():
    u = synth.uniform_f64(901, N)
    return {
        "sorted": np.sort(u),
        "reversed": np.sort(u)[::-1].copy(),
        "all_equal": np.full(N, 0.5),
        "four_values": np.floor(synth.uniform_f64(902, N) * 4.0) / 4.0,
        "organ_pipe": np.concatenate([np.sort(u[: N // 2]), np.sort(u[N // 2:])[::-1]]),
    }


@pytest.mark.parametrize("kind", ["sorted", "reversed", "all_equal", "four_values", "organ_pipe"])
def test_worst_case_inputs(kind):
    from paper_1107_3622_amd import ksort
    torch_dev()
    a = inputs()[kind]
    note(f"worst case {kind} n={N}")
    t = to_dev(a)
    ksort.ksort_profile_read()
    ksort.ksort_profile_enable(True)
    p = ksort.sort_(t)
    ksort.ksort_profile_enable(False)
    # level passes that had work (the host's last batch of launches may run
    # past the last one; those find nothing to do)
    levels = sum(1 for r in ksort.ksort_profile_read() if r["live_keys"] + r["finish_keys"] > 0)
    want, wp = oracle.sorted_copy(a)
    assert_bit_equal(to_host(t), want, kind)
    assert p == wp
    if kind in ("sorted", "reversed", "all_equal"):
        # every partition leaves one side empty and the other one key shorter:
        # levels 0 .. N-CUTOFF-1 partition, the last one finishes CUTOFF keys
        assert levels == N - CUTOFF + 1, levels
