"""GPU parity of the batched form: every array of a packed batch sorted
bit-exactly as the oracle sorts it alone, with its first pivot."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_bit_equal, note, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


def run(keys, offs, tune=None):
    from paper_1107_3622_amd import ksort
    t = to_dev(keys)
    fp = ksort.ksort_segmented(t, to_dev(offs), tune=tune)
    return to_host(t), to_host(fp)


def check(keys, offs, what, tune=None):
    note(f"{what} nseg={offs.size - 1} n={keys.size}")
    got, fp = run(keys, offs, tune)
    want = keys.copy()
    wfp = oracle.segmented_(want, offs)
    assert_bit_equal(got, want, what)
    assert np.array_equal(fp, wfp), f"{what}: first pivots differ at {np.flatnonzero(fp != wfp)[:5]}"


def test_all_permutations_up_to_8():
    torch_dev()
    arrays = [np.array(p, dtype=np.float64) for n in range(1, 9) for p in itertools.permutations(range(n))]
    offs = np.zeros(len(arrays) + 1, dtype=np.int64)
    np.cumsum([a.size for a in arrays], out=offs[1:])
    check(np.concatenate(arrays), offs, "all permutations n<=8")


def test_batched_small():
    keys, offs = synth.batched(9, 10, 256, 32, 65536)
    check(keys, offs, "batched 256 arrays")


def test_batched_f32_with_empty_and_single():
    torch_dev()
    lens = synth.loguniform_int(21, 300, 1, 20000)
    lens[::7] = 0
    lens[::11] = 1
    offs = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    keys = synth.uniform_f32(22, int(offs[-1]))
    check(keys, offs, "f32 with empty and one-key arrays")


def test_graph_replay_matches_each_time():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    keys, offs = synth.batched(9, 10, 512, 32, 65536)
    want = keys.copy()
    wfp = oracle.segmented_(want, offs)
    src = to_dev(keys)
    t = torch.empty_like(src)
    d_off = to_dev(offs)
    fp = torch.empty(offs.size - 1, dtype=torch.int64, device="cuda")
    for r in range(4):
        note(f"graph replay {r}")
        t.copy_(src)
        torch.cuda.synchronize()
        ksort.ksort_segmented(t, d_off, first_pivots=fp)
        assert_bit_equal(to_host(t), want, f"replay {r}")
        assert np.array_equal(to_host(fp), wfp)
        # eager work between replays
        (t * 2).sum().item()


def test_bad_offsets_rejected():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    t = torch.rand(100, dtype=torch.float64, device="cuda")
    for offs in ([0, 50, 40, 100], [0, 50, 101], [-1, 10]):
        note(f"bad offsets {offs}")
        with pytest.raises(ksort.KsortError):
            ksort.ksort_segmented(t, to_dev(np.array(offs, dtype=np.int64)))


def test_epoch_wrap_segmented(monkeypatch):
    # the recorded graph clears the look-back words at each wrap of the tags
    torch_dev()
    monkeypatch.setenv("KSORT_EPOCH_SPAN", "3")
    keys, offs = synth.batched(31, 32, 257, 32, 65536)
    check(keys, offs, "batched 257 arrays, tags wrap every 3 passes")


def test_c3_full_batch():
    # The batched workload itself: 4096 arrays, lengths log-uniform in
    # [32, 65536] (seed 9), keys from seed 10; every array and first pivot
    # against the oracle, recorded graph then replay.
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    keys, offs = synth.batched(9, 10, 4096, 32, 65536)
    want = keys.copy()
    wfp = oracle.segmented_(want, offs)
    src = to_dev(keys)
    d_off = to_dev(offs)
    for r in range(2):
        note(f"c3 batch of 4096 arrays, {keys.size} keys, run {r}")
        t = src.clone()
        fp = torch.empty(offs.size - 1, dtype=torch.int64, device="cuda")
        ksort.ksort_segmented(t, d_off, first_pivots=fp)
        assert_bit_equal(to_host(t), want, f"c3 run {r}")
        assert np.array_equal(to_host(fp), wfp), f"c3 run {r}: first pivots"
