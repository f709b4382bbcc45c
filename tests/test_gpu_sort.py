"""GPU parity: the HIP sort (through the C ABI) against the literal CPU
oracle, bit for bit, with the first partition's pivot index."""
import numpy as np
import pytest

import synth
from gpu_util import assert_bit_equal, note, oracle_sorted, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    torch_dev()
    from paper_1107_3622_amd import ksort
    ksort.load()
    return ksort


def gpu_sort(ks, a: np.ndarray, tune=None):
    t = to_dev(a)
    fp = ks.sort_(t, tune=tune)
    return to_host(t), fp


def check(ks, a, what, tune=None):
    note(f"{what} n={a.size} dtype={a.dtype} tune={tune}")
    got, fp = gpu_sort(ks, a, tune)
    want, wfp = oracle_sorted(a)
    assert_bit_equal(got, want, what)
    assert fp == wfp, f"{what}: first pivot {fp} != oracle {wfp}"


def test_illustration(ks):
    a = np.array([55, 66, 60, 78, 22, 50, 75, 5, 8, 94], dtype=np.float64)
    got, fp = gpu_sort(ks, a)
    assert list(got) == [5, 8, 22, 50, 55, 60, 66, 75, 78, 94]
    assert fp == 4
    got32, fp32 = gpu_sort(ks, a.astype(np.float32))
    assert list(got32) == [5, 8, 22, 50, 55, 60, 66, 75, 78, 94] and fp32 == 4


SIZES = [0, 1, 2, 3, 5, 63, 64, 65, 255, 256, 257, 1000, 2047, 2048, 2049, 2050, 4095, 4096, 4097,
         6000, 8191, 8192, 8193, 12289, 65537, 100_003, 250_001]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["uniform_f64", "uniform_f32"])
def test_sizes_bit_exact(ks, n, kind):
    a = synth.uniform_f64(500 + n, n) if kind == "uniform_f64" else synth.uniform_f32(500 + n, n)
    check(ks, a, f"{kind} n={n}")


def test_c0_n1e5(ks):
    check(ks, synth.make("c0_n1e5_f64"), "c0 n=1e5 seed 1")


def test_every_variant(ks):
    for dt, code in (("f64", ks.KSORT_F64), ("f32", ks.KSORT_F32)):
        a = synth.uniform_f64(31, 300_007) if dt == "f64" else synth.uniform_f32(31, 300_007)
        for variant in ks.ksort_variants(code):
            check(ks, a, f"variant {variant} {dt}", tune=variant)


def test_duplicates(ks):
    check(ks, synth.grid16_f64(8, 300_000), "2^16 grid n=3e5")
    # four distinct values: long runs of equal keys (one key per level)
    a = np.floor(synth.uniform_f64(9, 20_000) * 4).astype(np.float64)
    check(ks, a, "four values n=2e4")
    check(ks, np.full(9000, 0.25), "all equal n=9000")


def test_sorted_and_reversed(ks):
    a = np.sort(synth.uniform_f64(10, 12_000))
    check(ks, a, "sorted n=12000")
    check(ks, a[::-1].copy(), "reversed n=12000")


def test_special_values_order(ks):
    # infinities and subnormals sort like any other keys; no NaN, one zero sign
    a = synth.uniform_f64(11, 50_000) - 0.5
    a[::97] = np.inf
    a[::89] = -np.inf
    a[::83] = 5e-324
    a[a == 0] = 0.0
    a = np.where(a == 0, 0.0, a)
    check(ks, a, "infinities and subnormals")


def test_c1_headline_n7e6(ks):
    check(ks, synth.make("c1_n7e6_f64"), "c1 n=7e6 seed 4")


def test_repeat_is_deterministic(ks):
    torch = torch_dev()
    a = synth.uniform_f64(12, 1_000_000)
    want, wfp = oracle_sorted(a)
    src = to_dev(a)
    for r in range(5):
        note(f"repeat {r}")
        t = src.clone()
        fp = ks.sort_(t)
        assert fp == wfp
        assert torch.equal(t, to_dev(want))


def test_errors(ks):
    torch = torch_dev()
    t = torch.zeros(10, dtype=torch.float64, device="cuda")
    lib = ks.load()
    assert lib.ksort_f64(None, 10, None) == -1
    assert lib.ksort_f64(t.data_ptr(), -1, None) == -1
    assert lib.ksort_sort_ex(3, t.data_ptr(), 10, None, None, None) == -1
    with pytest.raises(ks.KsortError):
        ks.ksort_sort_ex(t, tune=(256, 3, 2048))
    with pytest.raises(TypeError):
        ks.ksort_f32(t)
    # output index arrays are checked before any device call: wrong type,
    # host memory or too few entries are refused, and the keys are untouched
    src = torch.arange(10, dtype=torch.float64, device="cuda").flip(0).contiguous()
    t = src.clone()
    for bad in (torch.zeros(1, dtype=torch.int64), torch.zeros(1, dtype=torch.int32, device="cuda"),
                torch.zeros(0, dtype=torch.int64, device="cuda")):
        with pytest.raises(ValueError):
            ks.ksort_sort_ex(t, first_pivot=bad)
    left = torch.tensor([0, 5], dtype=torch.int64, device="cuda")
    length = torch.tensor([5, 5], dtype=torch.int64, device="cuda")
    out = torch.zeros_like(t)
    with pytest.raises(ValueError):
        ks.ksort_partition_level(t, out, left, length, pivots=torch.zeros(1, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        ks.ksort_partition_level_exact(t, out, left, length, pivots=torch.zeros(2, dtype=torch.int64))
    offs = torch.tensor([0, 4, 10], dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        ks.ksort_segmented(t, offs, first_pivots=torch.zeros(1, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        ks.ksort_sort_exact(t, calls_cap=-1)
    assert torch.equal(t, src)


def test_lookback_wait_is_bounded(ks, monkeypatch):
    # A poll limit of 0 makes every tile that finds a predecessor's count not
    # yet published end the pass at once: the call reports KSORT_EINTERNAL
    # and every kernel exits normally.  With the limit restored the same
    # workspace sorts correctly again.
    torch = torch_dev()
    src = synth.torch_fill("uniform_f64", 4, 7_000_000, "cuda")
    ref = torch.sort(src)[0]
    monkeypatch.setenv("KSORT_SPIN_LIMIT", "0")
    raised = 0
    for r in range(3):
        note(f"spin limit 0, run {r}")
        t = src.clone()
        try:
            ks.ksort_f64(t)
        except ks.KsortError as e:
            raised += 1
            assert e.code == -10 and "timed out" in str(e)
        else:
            assert torch.equal(t, ref)
    assert raised >= 1
    monkeypatch.delenv("KSORT_SPIN_LIMIT")
    note("spin limit restored")
    t = src.clone()
    ks.ksort_f64(t)
    assert torch.equal(t, ref)


def test_small_arrays_take_the_small_variant(ks):
    # Without a caller default or a tuned bucket, arrays below 3e6 keys run
    # with 16 keys per thread and a 1024-key finish, larger ones with the
    # default variant; both sort exactly.
    torch = torch_dev()
    for n, want in ((1_000_000, (512, 16, 1024)), (4_000_000, ks.ksort_get_default(ks.KSORT_F64))):
        note(f"variant choice n={n}")
        src = synth.torch_fill("uniform_f64", 7, n, "cuda")
        t = src.clone()
        ks.ksort_profile_read()
        ks.ksort_profile_enable(True)
        ks.ksort_f64(t)
        ks.ksort_profile_enable(False)
        recs = ks.ksort_profile_read()
        assert {(r["block"], r["items"], r["cutoff"]) for r in recs} == {tuple(want)}
        assert torch.equal(t, torch.sort(src)[0])


def test_epoch_wrap_plain(ks, monkeypatch):
    # Look-back tags that wrap every 3 passes (KSORT_EPOCH_SPAN, read when a
    # sort starts): the words are cleared at each wrap, and the sorts stay
    # bit-exact, also on ordered input, where the passes number in thousands.
    monkeypatch.setenv("KSORT_EPOCH_SPAN", "3")
    check(ks, synth.uniform_f64(41, 1_000_000), "tags wrap every 3 passes, f64")
    check(ks, synth.uniform_f32(42, 250_001), "tags wrap every 3 passes, f32")
    check(ks, np.sort(synth.uniform_f64(43, 12_000)), "tags wrap every 3 passes, sorted input")


def bits_multiset(a: np.ndarray) -> np.ndarray:
    u = a.view(np.uint64 if a.dtype == np.float64 else np.uint32)
    return np.sort(u)


@pytest.mark.parametrize("n", [40, 100, 1500, 50_000, 600_000])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_nan_inputs_stay_a_permutation(ks, n, dt):
    # NaN is outside the bit-exact contract (a NaN compares false and goes
    # left), but the output must still hold every input key: the leaves that
    # place keys by rank order NaNs after the numbers.
    rng = np.random.default_rng(n)
    for frac in (0.01, 0.3, 1.0):
        a = rng.random(n).astype(dt)
        a[rng.random(n) < frac] = np.nan
        a[0] = np.nan if frac > 0.2 else a[0]  # a NaN as the first key
        note(f"NaN fraction {frac} n={n} {np.dtype(dt).name}")
        got, _ = gpu_sort(ks, a)
        assert np.array_equal(bits_multiset(got), bits_multiset(a)), f"n={n} frac={frac}: keys lost or duplicated"


def test_counter_tickets_sort_the_same(ks, monkeypatch):
    # KSORT_FIXED_FIRST=0: every work ticket of the library's own passes
    # comes from the counter (no reliance on the whole grid being resident);
    # the results are those of the default, for both key types and across
    # the variants' size ranges, and the plain batched call too.
    torch = torch_dev()
    monkeypatch.setenv("KSORT_FIXED_FIRST", "0")
    for kind, n in (("uniform_f64", 7_000_000), ("uniform_f64", 1_000_000), ("uniform_f32", 3_000_001)):
        note(f"counter tickets {kind} n={n}")
        src = synth.torch_fill(kind, 30 + n % 7, n, "cuda")
        t = src.clone()
        fp = ks.sort_(t)
        assert torch.equal(t, torch.sort(src)[0])
        assert fp == int((src[1:] < src[0]).sum().item())
    monkeypatch.delenv("KSORT_FIXED_FIRST")


def test_stream_copy(ks):
    # The streaming copy used as the bandwidth ceiling: every byte, for
    # sizes with and without a tail of less than 16 bytes, and the errors.
    torch = torch_dev()
    for nbytes in (16, 48, 17 * 16, (1 << 20) + 16 * 3, (64 << 20) + 16 * 5):
        note(f"stream copy {nbytes} bytes")
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        ks.ksort_stream_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
    for nbytes in (1, 15, 33, 1000003):
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        ks.ksort_stream_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src), nbytes
    big = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ks.KsortError):
        ks.ksort_stream_copy(big[1:17], big[32:48])  # not 16-byte aligned


def test_validate_refuses_inputs_outside_the_contract(ks, monkeypatch):
    # KSORT_VALIDATE=1: a NaN, or both zeros, make the call fail with
    # KSORT_EINVAL before any key moves; other inputs sort as usual.
    torch = torch_dev()
    monkeypatch.setenv("KSORT_VALIDATE", "1")
    for dt in (torch.float64, torch.float32):
        base = synth.torch_fill("uniform_f64", 41, 100_000, "cuda").to(dt)
        for what, pos, val in (("nan", 77_777, float("nan")), ("both zeros", None, None)):
            t = base.clone()
            if what == "nan":
                t[pos] = val
            else:
                t[10] = 0.0
                t[20] = -0.0
            keep = t.clone()
            note(f"validate {what} {dt}")
            with pytest.raises(ks.KsortError) as ei:
                ks.sort_(t)
            assert ei.value.code == -1 and "KSORT_VALIDATE" in str(ei.value)
            assert torch.equal(t.view(torch.int64 if dt == torch.float64 else torch.int32),
                               keep.view(torch.int64 if dt == torch.float64 else torch.int32))
        t = base.clone()
        t[5] = -0.0  # one kind of zero only: inside the contract
        ks.sort_(t)
        assert torch.equal(t, torch.sort(base.clone().index_fill_(0, torch.tensor([5], device="cuda"), -0.0))[0])
    monkeypatch.delenv("KSORT_VALIDATE")
