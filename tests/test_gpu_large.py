"""GPU parity at the full sizes of the large and duplicate-heavy workloads,
the autotuner, and the per-level profile records.

At 2^28 / 2^29 keys the literal oracle would take minutes, so the checks
there are properties that hold at any size: the output equals the library
sort of torch (the sorted arrangement is unique for keys without NaN and
with one sign of zero), and the first pivot equals the closed form
i = #{x : x < a[0]} (pinned against the literal oracle on the CPU)."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_bit_equal, note, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def check_by_properties(name):
    from paper_1107_3622_amd import ksort
    torch = torch_dev()
    note(f"{name} (torch.sort + closed-form pivot)")
    t = synth.torch_make(name, "cuda")
    want_pivot = int((t < t[0]).sum().item())
    ref = torch.sort(t)[0]
    p = ksort.sort_(t)
    assert torch.equal(t, ref), f"{name}: output differs from torch.sort"
    assert p == want_pivot, f"{name}: first pivot {p}, closed form {want_pivot}"
    del t, ref
    torch.cuda.empty_cache()


def test_c2_n2p28_f64():
    check_by_properties("c2_n2^28_f64")


def test_c2_n2p29_f32():
    check_by_properties("c2_n2^29_f32")


@pytest.mark.parametrize("name", ["c2_grid16_n1e7_f64", "c1_n1e7_f64", "c1_n2.5e6_f64", "c1_n1e6_f64"])
def test_oracle_full_size(name):
    from paper_1107_3622_amd import ksort
    torch_dev()
    a = synth.make(name)
    note(f"{name} vs oracle")
    t = to_dev(a)
    p = ksort.sort_(t)
    want, wp = oracle.sorted_copy(a)
    assert_bit_equal(to_host(t), want, name)
    assert p == wp


def test_autotune_then_sort():
    from paper_1107_3622_amd import ksort
    torch_dev()
    note("autotune f64 n=300000")
    best = ksort.ksort_autotune(ksort.KSORT_F64, 300_000)
    assert best in ksort.ksort_variants(ksort.KSORT_F64)
    a = synth.uniform_f64(77, 300_000)
    t = to_dev(a)
    p = ksort.sort_(t)  # now runs the tuned variant for this size
    want, wp = oracle.sorted_copy(a)
    ksort.ksort_tune_file(None)  # later tests take the untuned defaults
    assert_bit_equal(to_host(t), want, "after autotune")
    assert p == wp


def test_tuning_persists_in_a_json_file(tmp_path):
    # ksort_autotune_batch times every variant on copies of the caller's
    # batch (left as it is) and ksort_autotune on a seeded array; both
    # choices land in the JSON tuning file, and a new process that names the
    # file sorts with them.
    import json
    import subprocess
    import sys
    from paper_1107_3622_amd import ksort
    torch = torch_dev()
    path = tmp_path / "tune.json"
    ksort.ksort_tune_file(None)  # no choices from earlier tests
    ksort.ksort_tune_file(str(path))
    try:
        keys, offs = synth.batched(5, 6, 300, 32, 20000)
        t, d = to_dev(keys), to_dev(offs)
        note("autotune a batch of 300 arrays")
        best_b = ksort.ksort_autotune_batch(t, d)
        assert torch.equal(t, to_dev(keys)), "the caller's batch is left as it is"
        note("autotune f32 n=200000")
        best_s = ksort.ksort_autotune(ksort.KSORT_F32, 200_000)
        entries = json.load(open(path))["entries"]
        kinds = {(e["kind"], e["dtype"]): (e["block"], e["items"], e["cutoff"]) for e in entries}
        assert kinds[("batch", 0)] == best_b and kinds[("single", 1)] == best_s
        assert all(e["arch"].startswith("gfx950") and e["ms"] > 0 and e["default_ms"] > 0 for e in entries)
        assert ksort.ksort_tune_count() == len(entries) == 2
        code = (
            "import sys; sys.path.insert(0, %r); import torch, synth; from paper_1107_3622_amd import ksort;"
            "ksort.ksort_tune_file(%r);"
            "k, o = synth.batched(5, 6, 300, 32, 20000); t = torch.from_numpy(k).cuda(); d = torch.from_numpy(o).cuda();"
            "ksort.ksort_profile_enable(True); ksort.ksort_segmented(t, d); ksort.ksort_profile_enable(False);"
            "r = ksort.ksort_profile_read(); print(r[0]['block'], r[0]['items'], r[0]['cutoff'])"
        ) % (ROOT, str(path))
        note("a new process reads the tuning file")
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0, out.stderr[-2000:]
        assert tuple(int(x) for x in out.stdout.split()[-3:]) == best_b
    finally:
        ksort.ksort_tune_file(None)
    assert ksort.ksort_tune_count() == 0


def test_profile_records_account_for_every_key():
    from paper_1107_3622_amd import ksort
    torch_dev()
    n = 1_000_000
    a = synth.uniform_f64(2, n)
    t = to_dev(a)
    note("profiled sort n=1e6")
    ksort.ksort_profile_read()
    ksort.ksort_profile_enable(True)
    ksort.ksort_f64(t)
    ksort.ksort_profile_enable(False)
    recs = ksort.ksort_profile_read()
    assert recs and all(r["ms"] > 0 for r in recs)
    assert [r["stage"] for r in recs] == list(range(len(recs)))
    assert recs[0]["live_keys"] == n
    # each partition places its key; every other key ends in a finish
    # segment or as a one-key side, so the keys finished never exceed n and
    # the partitions (one key each) plus the finished keys cover all n keys
    fin = sum(r["finish_keys"] for r in recs)
    assert 0 < fin <= n
    # passes that partition come first: a pass with nothing to partition lists
    # no segment for the next one.  (A chain of one-tile segments is
    # partitioned within one pass, so the keys partitioned per pass need not
    # shrink.)  Pass 0 partitions every key once.
    live = [r["live_keys"] for r in recs]
    k0 = next((k for k, v in enumerate(live) if v == 0), len(live))
    assert all(v == 0 for v in live[k0:])
    assert sum(live) >= n
    assert_bit_equal(to_host(t), np.sort(a), "profiled sort")
