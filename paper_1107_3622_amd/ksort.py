"""Python binding of libksort.so (ctypes).

Argument marshalling only: every step of the sort runs in the HIP library.
Tensors are torch tensors on the HIP device (PyTorch supplies device memory
and streams); each function passes their data pointers and the current
stream to the C entry point of the same name and raises KsortError on a
negative return code.  There is no fallback: if the library is not built,
or no gfx950 device is present, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libksort.so")

KSORT_F64 = 0
KSORT_F32 = 1

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_p = ctypes.c_void_p
_int = ctypes.c_int


class KsortError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where} failed with {code}: {detail}")
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("block", _i32), ("items", _i32), ("cutoff", _i32), ("reserved", _i32)]

    def as_tuple(self):
        return (self.block, self.items, self.cutoff)


class LevelRecord(ctypes.Structure):
    _fields_ = [("call", _i64), ("dtype", _i32), ("stage", _i32), ("live_keys", _i64),
                ("finish_keys", _i64), ("ms", ctypes.c_double), ("block", _i32), ("items", _i32),
                ("cutoff", _i32), ("grid", _i32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class RequestInfo(ctypes.Structure):
    _fields_ = [("n", _i64), ("dtype", _i32), ("state", _i32), ("first_pivot", _i64),
                ("t_submit_s", ctypes.c_double), ("t_admit_s", ctypes.c_double),
                ("t_done_s", ctypes.c_double), ("levels", _i32), ("pad", _i32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("admitted", _i64), ("completed", _i64), ("rejected", _i64),
                ("cancelled", _i64), ("failed", _i64), ("keys_completed", _i64), ("ticks", _i64),
                ("busy_s", ctypes.c_double), ("p50_latency_s", ctypes.c_double),
                ("p99_latency_s", ctypes.c_double), ("mean_latency_s", ctypes.c_double),
                ("inflight_now", _i64), ("queued_now", _i64), ("budget_used_bytes", _i64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes)
SIGNATURES = {
    "ksort_f64": (_int, [_p, _i64, _p]),
    "ksort_f32": (_int, [_p, _i64, _p]),
    "ksort_sort_ex": (_int, [_int, _p, _i64, _p, _p, _p]),
    "ksort_sort_static": (_int, [_int, _p, _i64, _p, _p]),
    "ksort_partition_level": (_int, [_int, _p, _p, _i64, _p, _p, _i64, _p, _p]),
    "ksort_segmented": (_int, [_int, _p, _i64, _p, _i64, _p, _p, _p]),
    "ksort_partition_level_exact": (_int, [_int, _p, _p, _i64, _p, _p, _i64, _p, _p]),
    "ksort_sort_exact": (_int, [_int, _p, _i64, _p, _p, _i64, _p, _p]),
    "ksort_variants": (_int, [_int, _p, _int]),
    "ksort_get_default": (_int, [_int, _p]),
    "ksort_set_default": (_int, [_int, _p]),
    "ksort_autotune": (_int, [_int, _i64, _p, _p]),
    "ksort_autotune_batch": (_int, [_int, _p, _i64, _p, _i64, _p, _p]),
    "ksort_tune_file": (_int, [ctypes.c_char_p]),
    "ksort_tune_count": (_int, []),
    "ksort_profile_enable": (_int, [_int]),
    "ksort_profile_count": (_i64, []),
    "ksort_profile_read": (_i64, [_p, _i64]),
    "ksort_workspace_bytes": (ctypes.c_size_t, [_int, _i64, _i64]),
    "ksort_stream_copy": (_int, [_p, _p, ctypes.c_size_t, _int, _p]),
    "ksort_set_workspace": (_int, [_p, ctypes.c_size_t, _p]),
    "ksort_release_workspaces": (_int, []),
    "ksort_server_create": (_p, [ctypes.c_size_t, _int, _int]),
    "ksort_server_submit": (_int, [_p, _int, _p, _i64, ctypes.POINTER(ctypes.c_uint64)]),
    "ksort_server_poll": (_int, [_p, ctypes.c_uint64, ctypes.POINTER(_int)]),
    "ksort_server_wait": (_int, [_p, ctypes.c_uint64, ctypes.c_double]),
    "ksort_server_cancel": (_int, [_p, ctypes.c_uint64]),
    "ksort_server_result": (_int, [_p, ctypes.c_uint64, _p]),
    "ksort_server_stats": (_int, [_p, _p]),
    "ksort_server_destroy": (None, [_p]),
    "ksort_strerror": (ctypes.c_char_p, [_int]),
    "ksort_last_error": (ctypes.c_char_p, []),
    "ksort_version": (ctypes.c_char_p, []),
}

_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libksort.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_1107_3622_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def _check(rc: int, where: str) -> None:
    if rc < 0:
        lib = load()
        raise KsortError(rc, where, lib.ksort_last_error().decode(errors="replace") or
                         lib.ksort_strerror(rc).decode())


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return KSORT_F64
    if t.dtype == torch.float32:
        return KSORT_F32
    raise TypeError(f"keys must be float64 or float32, got {t.dtype}")


def _check_keys(t) -> None:
    if not t.is_cuda:
        raise ValueError("keys must live on the HIP device")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError("keys must be a 1-D contiguous tensor")


def _check_index_out(t, need: int, what: str) -> None:
    """An int64 output array on the device with room for `need` entries."""
    torch = _torch()
    if t.dtype != torch.int64 or not t.is_cuda or not t.is_contiguous() or t.numel() < need:
        raise ValueError(f"{what} must be a contiguous int64 device tensor of at least {need} entries")


def _tuning(tune) -> Optional[Tuning]:
    if tune is None:
        return None
    if isinstance(tune, Tuning):
        return tune
    b, i, c = tune
    return Tuning(b, i, c, 0)


def _ref(x):
    return ctypes.byref(x) if x is not None else None


def ksort_f64(t, stream=None) -> None:
    """Sort a float64 device tensor in place."""
    _check_keys(t)
    if _dtype_code(t) != KSORT_F64:
        raise TypeError("ksort_f64 needs float64 keys")
    _check(load().ksort_f64(t.data_ptr(), t.numel(), _stream(stream)), "ksort_f64")


def ksort_f32(t, stream=None) -> None:
    """Sort a float32 device tensor in place."""
    _check_keys(t)
    if _dtype_code(t) != KSORT_F32:
        raise TypeError("ksort_f32 needs float32 keys")
    _check(load().ksort_f32(t.data_ptr(), t.numel(), _stream(stream)), "ksort_f32")


def ksort_sort_ex(t, first_pivot=None, tune=None, stream=None) -> None:
    """Sort in place; `first_pivot` (int64 device tensor of 1) receives the
    index at which the first partition left a[0]."""
    _check_keys(t)
    if first_pivot is not None:
        _check_index_out(first_pivot, 1, "first_pivot")
    fp = first_pivot.data_ptr() if first_pivot is not None else None
    tn = _tuning(tune)
    _check(load().ksort_sort_ex(_dtype_code(t), t.data_ptr(), t.numel(), fp, _ref(tn), _stream(stream)),
           "ksort_sort_ex")


def ksort_sort_static(t, first_pivot=None, stream=None) -> None:
    """Sort in place with the library's static scratch (no allocation)."""
    _check_keys(t)
    if first_pivot is not None:
        _check_index_out(first_pivot, 1, "first_pivot")
    fp = first_pivot.data_ptr() if first_pivot is not None else None
    _check(load().ksort_sort_static(_dtype_code(t), t.data_ptr(), t.numel(), fp, _stream(stream)),
           "ksort_sort_static")


def sort_(t, tune=None, stream=None) -> int:
    """Sort in place and return the first partition's pivot index."""
    torch = _torch()
    fp = torch.empty(1, dtype=torch.int64, device=t.device)
    ksort_sort_ex(t, fp, tune, stream)
    return int(fp.item())


def ksort_partition_level(d_in, d_out, seg_left, seg_len, pivots=None, stream=None):
    """One partition (Steps 1-4) of each segment from d_in into d_out.
    Returns the int64 device tensor of pivot indices."""
    torch = _torch()
    _check_keys(d_in)
    _check_keys(d_out)
    if d_in.dtype != d_out.dtype or d_in.numel() != d_out.numel():
        raise ValueError("d_in and d_out must have the same dtype and size")
    for s in (seg_left, seg_len):
        if s.dtype != torch.int64 or not s.is_cuda or not s.is_contiguous():
            raise ValueError("segment arrays must be contiguous int64 device tensors")
    nseg = seg_left.numel()
    if seg_len.numel() != nseg:
        raise ValueError("seg_left and seg_len differ in length")
    if pivots is None:
        pivots = torch.empty(nseg, dtype=torch.int64, device=d_in.device)
    else:
        _check_index_out(pivots, nseg, "pivots")
    _check(load().ksort_partition_level(_dtype_code(d_in), d_in.data_ptr(), d_out.data_ptr(), d_in.numel(),
                                        seg_left.data_ptr(), seg_len.data_ptr(), nseg, pivots.data_ptr(),
                                        _stream(stream)), "ksort_partition_level")
    return pivots


def ksort_partition_level_exact(d_in, d_out, seg_left, seg_len, pivots=None, stream=None):
    """One partition (Steps 1-4) of each segment from d_in into d_out, leaving
    exactly the arrangement of the paper's sequential steps.  Returns the
    int64 device tensor of pivot indices."""
    torch = _torch()
    _check_keys(d_in)
    _check_keys(d_out)
    if d_in.dtype != d_out.dtype or d_in.numel() != d_out.numel():
        raise ValueError("d_in and d_out must have the same dtype and size")
    for s in (seg_left, seg_len):
        if s.dtype != torch.int64 or not s.is_cuda or not s.is_contiguous():
            raise ValueError("segment arrays must be contiguous int64 device tensors")
    nseg = seg_left.numel()
    if seg_len.numel() != nseg:
        raise ValueError("seg_left and seg_len differ in length")
    if pivots is None:
        pivots = torch.empty(nseg, dtype=torch.int64, device=d_in.device)
    else:
        _check_index_out(pivots, nseg, "pivots")
    _check(load().ksort_partition_level_exact(_dtype_code(d_in), d_in.data_ptr(), d_out.data_ptr(), d_in.numel(),
                                              seg_left.data_ptr(), seg_len.data_ptr(), nseg, pivots.data_ptr(),
                                              _stream(stream)), "ksort_partition_level_exact")
    return pivots


def ksort_sort_exact(t, calls_cap: int = 0, stream=None):
    """Steps 1-6 on t in place, every call leaving the literal arrangement.
    Returns (first pivot, total calls, (calls_cap', 3) int64 device tensor of
    (left, right, i) per call in no particular order, or None)."""
    torch = _torch()
    _check_keys(t)
    if calls_cap < 0:
        raise ValueError("calls_cap must be >= 0")
    fp = torch.empty(1, dtype=torch.int64, device=t.device)
    nc = torch.zeros(1, dtype=torch.int64, device=t.device)
    calls = torch.empty((max(calls_cap, 1), 3), dtype=torch.int64, device=t.device) if calls_cap > 0 else None
    _check(load().ksort_sort_exact(_dtype_code(t), t.data_ptr(), t.numel(), fp.data_ptr(),
                                   calls.data_ptr() if calls is not None else None, calls_cap,
                                   nc.data_ptr(), _stream(stream)), "ksort_sort_exact")
    ncalls = int(nc.item())
    if calls is not None:
        calls = calls[:min(ncalls, calls_cap)]
    return int(fp.item()), ncalls, calls


def ksort_segmented(t, offsets, first_pivots=None, tune=None, stream=None, want_pivots=True):
    """Sort every array t[offsets[u]:offsets[u+1]] in place.  Returns the int64
    device tensor of first pivots (relative), or None if not wanted."""
    torch = _torch()
    _check_keys(t)
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 device tensor")
    nseg = offsets.numel() - 1
    if nseg < 0:
        raise ValueError("offsets needs at least one entry")
    if first_pivots is None and want_pivots:
        first_pivots = torch.empty(max(nseg, 1), dtype=torch.int64, device=t.device)
    elif first_pivots is not None:
        _check_index_out(first_pivots, nseg, "first_pivots")
    fp = first_pivots.data_ptr() if first_pivots is not None else None
    tn = _tuning(tune)
    _check(load().ksort_segmented(_dtype_code(t), t.data_ptr(), t.numel(), offsets.data_ptr(), nseg, fp,
                                  _ref(tn), _stream(stream)), "ksort_segmented")
    return first_pivots[:nseg] if first_pivots is not None else None


def ksort_variants(dtype: int) -> list[tuple[int, int, int]]:
    lib = load()
    n = lib.ksort_variants(dtype, None, 0)
    _check(n, "ksort_variants")
    arr = (Tuning * max(n, 1))()
    lib.ksort_variants(dtype, arr, n)
    return [arr[j].as_tuple() for j in range(n)]


def ksort_get_default(dtype: int) -> tuple[int, int, int]:
    t = Tuning()
    _check(load().ksort_get_default(dtype, ctypes.byref(t)), "ksort_get_default")
    return t.as_tuple()


def ksort_set_default(dtype: int, tune: Optional[Sequence[int]]) -> None:
    tn = _tuning(tune)
    _check(load().ksort_set_default(dtype, _ref(tn)), "ksort_set_default")


def ksort_autotune(dtype: int, n: int, stream=None) -> tuple[int, int, int]:
    t = Tuning()
    _check(load().ksort_autotune(dtype, n, ctypes.byref(t), _stream(stream)), "ksort_autotune")
    return t.as_tuple()


def ksort_autotune_batch(t, offsets, stream=None) -> tuple[int, int, int]:
    """Tune the variant for packed batches like t (arrays per offsets); t is
    left as it is."""
    torch = _torch()
    _check_keys(t)
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 device tensor")
    tn = Tuning()
    _check(load().ksort_autotune_batch(_dtype_code(t), t.data_ptr(), t.numel(), offsets.data_ptr(),
                                       offsets.numel() - 1, ctypes.byref(tn), _stream(stream)),
           "ksort_autotune_batch")
    return tn.as_tuple()


def ksort_tune_file(path) -> None:
    """Persist tuning choices in the JSON file `path` (and apply its entries)."""
    _check(load().ksort_tune_file(None if path is None else os.fsencode(path)), "ksort_tune_file")


def ksort_tune_count() -> int:
    return int(load().ksort_tune_count())


def ksort_profile_enable(on: bool) -> None:
    _check(load().ksort_profile_enable(1 if on else 0), "ksort_profile_enable")


def ksort_profile_read() -> list[dict]:
    lib = load()
    n = lib.ksort_profile_count()
    arr = (LevelRecord * max(n, 1))()
    got = lib.ksort_profile_read(arr, n)
    return [arr[j].as_dict() for j in range(got)]


def ksort_stream_copy(dst, src, grid: int = 0, stream=None) -> None:
    """Copy src into dst (same size, device tensors) with the library's
    streaming copy kernel, the ceiling a level pass is measured against."""
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("dst and src must be contiguous device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    _check(load().ksort_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, grid, _stream(stream)),
           "ksort_stream_copy")


def ksort_workspace_bytes(dtype: int, n: int, nseg: int = 1) -> int:
    return int(load().ksort_workspace_bytes(dtype, n, nseg))


_user_ws: dict = {}  # stream handle -> tensor given to ksort_set_workspace (kept alive)


def ksort_set_workspace(buf, stream=None) -> None:
    """Scratch of calls on `stream` comes from `buf` (a contiguous uint8
    device tensor), or from the library's own memory again for None."""
    torch = _torch()
    s = _stream(stream)
    if buf is None:
        _check(load().ksort_set_workspace(None, 0, s), "ksort_set_workspace")
        _user_ws.pop(s, None)
        return
    if buf.dtype != torch.uint8 or not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("the workspace must be a contiguous uint8 device tensor")
    _check(load().ksort_set_workspace(buf.data_ptr(), buf.numel(), s), "ksort_set_workspace")
    _user_ws[s] = buf


def ksort_release_workspaces() -> None:
    _check(load().ksort_release_workspaces(), "ksort_release_workspaces")
    _user_ws.clear()


def ksort_version() -> str:
    return load().ksort_version().decode()


class Server:
    """Continuous-batching sort server (ksort_server_* entry points)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 256, device: int = 0):
        lib = load()
        h = lib.ksort_server_create(hbm_budget_bytes, max_inflight, device)
        if not h:
            raise KsortError(-1, "ksort_server_create", lib.ksort_last_error().decode())
        self._h = h
        self._keep = {}

    def submit(self, t) -> int:
        """Submit t for sorting in place.  The server works on streams of its
        own, so the current stream (which produced t) is synchronized first."""
        _check_keys(t)
        _torch().cuda.current_stream(t.device).synchronize()
        tk = ctypes.c_uint64()
        _check(load().ksort_server_submit(self._h, _dtype_code(t), t.data_ptr(), t.numel(), ctypes.byref(tk)),
               "ksort_server_submit")
        self._keep[tk.value] = t
        return tk.value

    def poll(self, ticket: int) -> int:
        st = _int()
        _check(load().ksort_server_poll(self._h, ticket, ctypes.byref(st)), "ksort_server_poll")
        return st.value

    def wait(self, ticket: int, timeout_s: float = -1.0) -> int:
        return load().ksort_server_wait(self._h, ticket, timeout_s)

    def cancel(self, ticket: int) -> int:
        return load().ksort_server_cancel(self._h, ticket)

    def result(self, ticket: int) -> dict:
        info = RequestInfo()
        _check(load().ksort_server_result(self._h, ticket, ctypes.byref(info)), "ksort_server_result")
        return info.as_dict()

    def release(self, ticket: int) -> None:
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        s = ServerStats()
        _check(load().ksort_server_stats(self._h, ctypes.byref(s)), "ksort_server_stats")
        return s.as_dict()

    def close(self) -> None:
        if self._h:
            load().ksort_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
