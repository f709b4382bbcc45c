"""The entry point that allocates nothing, ksort_sort_static (scratch in a
static device array), against the workspace entry point ksort_sort_ex, both
called through the C ABI: bit-equal keys and equal first pivots on two calls
in a row, the second with a smaller input, for both key types; sizes beyond
the static scratch are refused before any device work."""
import ctypes

import pytest

import synth
from gpu_util import note, torch_dev

pytestmark = pytest.mark.gpu

KSORT_ETOOLARGE = -5
MAX_KEYS = {0: 7_835_072, 1: 14_909_568}


def bits(torch, t):
    return t.view(torch.int64) if t.dtype == torch.float64 else t.view(torch.int32)


def compare(lib, torch, src, what):
    code = 0 if src.dtype == torch.float64 else 1
    n = src.numel()
    stream = torch.cuda.current_stream().cuda_stream
    a, b = src.clone(), src.clone()
    fa = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    fb = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    note(f"{what}: n={n} dtype={code}")
    assert lib.ksort_sort_ex(code, a.data_ptr(), n, fa.data_ptr(), None, stream) == 0, lib.ksort_last_error()
    rc = lib.ksort_sort_static(code, b.data_ptr(), n, fb.data_ptr(), stream)
    assert rc == 0, lib.ksort_last_error()
    torch.cuda.synchronize()
    assert torch.equal(bits(torch, a), bits(torch, b)), f"{what}: keys differ"
    assert int(fa.item()) == int(fb.item()), f"{what}: first pivot {int(fb.item())} != {int(fa.item())}"


def test_static_scratch_entry_point_matches_the_workspace_one():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    lib = ksort.load()
    for kind, sizes in (("uniform_f64", (7_000_000, 250_001)), ("uniform_f32", (MAX_KEYS[1], 65_537)),
                        ("grid16_f64", (MAX_KEYS[0], 3_001))):
        for k, n in enumerate(sizes):
            src = synth.torch_fill(kind, 900 + n, n, "cuda")
            compare(lib, torch, src, f"{kind} call {k + 1}")
    for n in (0, 1, 2, 64, 2048, 2049):
        compare(lib, torch, synth.torch_fill("uniform_f64", 950 + n, n, "cuda"), "small")


def test_static_scratch_refuses_larger_sorts():
    torch = torch_dev()
    from paper_1107_3622_amd import ksort
    lib = ksort.load()
    for code, dt in ((0, torch.float64), (1, torch.float32)):
        n = MAX_KEYS[code] + 1
        src = torch.rand(n, dtype=torch.float64, device="cuda").to(dt)
        t = src.clone()
        note(f"static scratch: n={n} beyond the limit, dtype={code}")
        rc = lib.ksort_sort_static(code, t.data_ptr(), n, None, torch.cuda.current_stream().cuda_stream)
        assert rc == KSORT_ETOOLARGE
        assert f"at most {MAX_KEYS[code]} keys" in lib.ksort_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(t, src), "a refused call leaves the keys alone"
    # the entry point still works after a refusal
    compare(lib, torch, synth.torch_fill("uniform_f64", 77, 123_457, "cuda"), "after a refusal")
