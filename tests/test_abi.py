"""The C-ABI library loads and exports every entry point include/ksort.h
declares; host-only entry points answer without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ksort.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"KSORT_API\s+[\w\s\*]+?\b(ksort_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1107_3622_amd import ksort
    if not os.path.exists(ksort.LIB_PATH):
        from paper_1107_3622_amd import build
        build.build()
    return ksort.load()


def test_header_declares_the_planned_surface():
    syms = declared_symbols()
    for s in ("ksort_f64", "ksort_f32", "ksort_sort_ex", "ksort_partition_level", "ksort_segmented",
              "ksort_server_create", "ksort_server_submit", "ksort_server_wait", "ksort_server_destroy",
              "ksort_strerror", "ksort_last_error", "ksort_autotune"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert missing == []


def test_binding_covers_every_symbol():
    from paper_1107_3622_amd import ksort
    assert sorted(ksort.SIGNATURES) == declared_symbols()


def test_host_only_calls(lib):
    assert lib.ksort_version().decode().startswith("ksort")
    assert lib.ksort_strerror(0) == b"ok"
    assert lib.ksort_strerror(-1) == b"invalid argument"
    from paper_1107_3622_amd import ksort
    v64 = ksort.ksort_variants(ksort.KSORT_F64)
    v32 = ksort.ksort_variants(ksort.KSORT_F32)
    for v in [(512, 24, 2048), (512, 16, 2048), (1024, 8, 2048), (512, 16, 1024)]:
        assert v in v64 and v in v32
    assert ksort.ksort_get_default(ksort.KSORT_F64) == (512, 24, 2048)
    assert (512, 32, 2048) in v32
    assert ksort.ksort_get_default(ksort.KSORT_F32) == (512, 32, 2048)
    assert lib.ksort_variants(7, None, 0) == -1
    # workspace: scratch of n keys plus descriptors, grows with n
    b1 = ksort.ksort_workspace_bytes(ksort.KSORT_F64, 1_000_000)
    b2 = ksort.ksort_workspace_bytes(ksort.KSORT_F64, 2_000_000)
    assert 8_000_000 < b1 < b2
    assert ksort.ksort_workspace_bytes(5, 10, 1) == 0
    assert ksort.ksort_workspace_bytes(ksort.KSORT_F64, 0, 1) > 0
    # caller memory: misaligned or too small is refused before any device call
    assert lib.ksort_set_workspace(8, 1 << 20, None) == -1
    assert lib.ksort_set_workspace(256, 1000, None) == -1
    # the literal-arrangement entry points check their arguments before any
    # device call
    assert lib.ksort_sort_exact(9, None, 0, None, None, 0, None, None) == -1
    assert lib.ksort_sort_exact(0, None, 1 << 31, None, None, 0, None, None) == -1
    assert lib.ksort_sort_exact(0, None, 5, None, None, 0, None, None) == -1
    assert lib.ksort_partition_level_exact(9, None, None, 10, None, None, 1, None, None) == -1
    assert lib.ksort_partition_level_exact(0, None, None, 1 << 31, None, None, 1, None, None) == -1
    assert lib.ksort_partition_level_exact(0, None, None, 10, None, None, 0, None, None) == 0


def test_set_default_rejects_unknown_variant(lib):
    from paper_1107_3622_amd import ksort
    with pytest.raises(ksort.KsortError):
        ksort.ksort_set_default(ksort.KSORT_F64, (256, 3, 2048))
    ksort.ksort_set_default(ksort.KSORT_F64, (1024, 8, 2048))
    assert ksort.ksort_get_default(ksort.KSORT_F64) == (1024, 8, 2048)
    ksort.ksort_set_default(ksort.KSORT_F64, None)
    assert ksort.ksort_get_default(ksort.KSORT_F64) == (512, 24, 2048)


def test_product_path_has_no_cpu_fallback():
    # the binding must not import the oracle or any CPU sort
    pkg = os.path.join(ROOT, "paper_1107_3622_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src
            assert "np.sort" not in src and "torch.sort" not in src


def test_tune_file_is_read_without_a_gpu(lib, tmp_path):
    # the tuning file's entries are read on the host; lines that are not a
    # whole entry are skipped; NULL forgets every choice
    p = tmp_path / "tune.json"
    p.write_text(
        '{"version": 1, "entries": [\n'
        '{"arch": "gfx950", "kind": "batch", "dtype": 0, "bucket": 25, "block": 512, "items": 16, '
        '"cutoff": 1024, "ms": 1.5, "default_ms": 2.0},\n'
        '{"arch": "gfx942", "kind": "single", "dtype": 1, "bucket": 20, "block": 512, "items": 32, '
        '"cutoff": 2048, "ms": 0.5, "default_ms": 0.5},\n'
        '{"arch": "gfx950", "kind": "single", "dtype": 0},\n'
        ']}\n')
    assert lib.ksort_tune_file(str(p).encode()) == 0
    assert lib.ksort_tune_count() == 2
    assert lib.ksort_tune_file(str(p).encode()) == 0  # read again: the same entries replace themselves
    assert lib.ksort_tune_count() == 2
    assert lib.ksort_tune_file(None) == 0
    assert lib.ksort_tune_count() == 0
    assert lib.ksort_tune_file(str(tmp_path / "missing.json").encode()) == 0
    assert lib.ksort_tune_count() == 0
    assert lib.ksort_tune_file(None) == 0
