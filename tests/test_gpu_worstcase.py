"""K-sort's worst cases on the GPU (the paper's average-case analysis,
Sections 1 and 4, assumes i.i.d. keys; ordered inputs and heavy duplicates
make every partition peel off a single key): sorted, reverse-sorted,
all-equal and few-distinct inputs sort bit-exactly as the oracle sorts
them, and the keys partitioned add up to what Steps 1-6 imply."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_bit_equal, note, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

N = 20_000


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
    recs = ksort.ksort_profile_read()
    # level passes that had work (the host's last batch of launches may run
    # past the last one; those find nothing to do)
    levels = sum(1 for r in recs if r["live_keys"] + r["finish_keys"] > 0)
    cutoff = recs[0]["cutoff"]  # the LDS finish size of the variant that ran
    partitioned = sum(r["live_keys"] for r in recs)
    finished = sum(r["finish_keys"] for r in recs)
    want, wp = oracle.sorted_copy(a)
    assert_bit_equal(to_host(t), want, kind)
    assert p == wp
    if kind in ("sorted", "reversed", "all_equal"):
        # every partition leaves one side empty and the other one key shorter:
        # segments of N, N-1, ..., cutoff+1 keys are partitioned, one each,
        # and the last cutoff keys are finished in LDS.  A chain of one-tile
        # segments runs within one pass, so the passes number at most one
        # per partition plus the finish.
        assert partitioned == sum(range(cutoff + 1, N + 1)), partitioned
        assert finished == cutoff, finished
        assert levels <= N - cutoff + 1, levels
