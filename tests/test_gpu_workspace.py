"""GPU parity of calls whose scratch lives in caller memory
(ksort_set_workspace): the same results as with library memory, a call that
needs more than the given memory fails before touching the keys, and the
stream returns to library memory afterwards."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_bit_equal, note, oracle_sorted, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


def test_sorts_in_caller_memory():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    n = 1_000_000
    need = ksort.ksort_workspace_bytes(ksort.KSORT_F64, n, 4096)
    buf = torch.full((need,), 0xA5, dtype=torch.uint8, device="cuda")
    note(f"workspace of {need} bytes for n={n}")
    ksort.ksort_set_workspace(buf)
    try:
        # plain sorts (three inputs) with the first pivot
        for seed in (31, 32, 33):
            a = synth.uniform_f64(seed, n)
            t = to_dev(a)
            fp = ksort.sort_(t)
            want, wfp = oracle_sorted(a)
            assert_bit_equal(to_host(t), want, f"sort in caller memory, seed {seed}")
            assert fp == wfp
        assert int((buf != 0xA5).sum()) > 0  # the library wrote into the given memory
        # a segmented batch of the same total size
        lens = synth.loguniform_int(34, 1500, 32, 2000)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        a = synth.uniform_f64(35, int(offs[-1]))
        t = to_dev(a)
        note(f"segmented in caller memory, {offs[-1]} keys")
        fps = to_host(ksort.ksort_segmented(t, to_dev(offs)))
        b = a.copy()
        wfps = oracle.segmented_(b, offs)
        assert_bit_equal(to_host(t), b, "segmented in caller memory")
        assert np.array_equal(fps, wfps)
        # one partition level
        left = np.array([0, 400_000], dtype=np.int64)
        length = np.array([300_000, 600_000], dtype=np.int64)
        a = synth.uniform_f64(36, n)
        out = torch.zeros(n, dtype=torch.float64, device="cuda")
        note("partition level in caller memory")
        piv = to_host(ksort.ksort_partition_level(to_dev(a), out, to_dev(left), to_dev(length)))
        b = a.copy()
        assert np.array_equal(piv, oracle.partition_level_(b, left, length))
        # a call that needs more than the given memory fails and leaves the
        # keys as they were
        big = synth.uniform_f64(37, 4 * n)
        t = to_dev(big)
        note("call larger than the workspace")
        with pytest.raises(ksort.KsortError) as e:
            ksort.ksort_f64(t)
        assert e.value.code == -2
        assert_bit_equal(to_host(t), big, "keys untouched after the refused call")
    finally:
        ksort.ksort_set_workspace(None)
    # library memory again: the larger call works
    note("library memory again")
    ksort.ksort_f64(t)
    assert torch.equal(t, torch.sort(to_dev(big))[0])


def test_workspace_arguments():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    lib = ksort.load()
    buf = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    assert lib.ksort_set_workspace(buf.data_ptr() + 8, 4096, None) == -1   # misaligned
    assert lib.ksort_set_workspace(buf.data_ptr(), 1024, None) == -1       # too small
    with pytest.raises(ValueError):
        ksort.ksort_set_workspace(torch.empty(8192, dtype=torch.float32, device="cuda"))
    # a tiny workspace: a small sort fits, a larger one is refused
    ksort.ksort_set_workspace(buf)
    try:
        a = synth.uniform_f64(38, 1000)
        t = to_dev(a)
        ksort.ksort_f64(t)
        assert np.array_equal(to_host(t), np.sort(a))
        t = to_dev(synth.uniform_f64(39, 100_000))
        with pytest.raises(ksort.KsortError):
            ksort.ksort_f64(t)
    finally:
        ksort.ksort_set_workspace(None)
