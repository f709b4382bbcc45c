"""K-sort CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Python access (ctypes + numpy) to the literal C oracle in ``ksort_oracle.c``:
K-sort of arXiv 1107.3622, Section 1.1, Steps 1-6, with the Step-3.1
temp/flag handling, in double and float.  Only the test suite, the package
smoke check and the benchmark's CPU-baseline leg may import this module; the
HIP library never links or calls it and the two share no code.

Pins: the CPU test suite checks this oracle against the Section 1.2
illustration, brute force over every permutation of n <= 8 and small
multisets, closed forms for the pivot index and the one-level arrangement,
the exact mean comparison count of Quick sort (Knuth vol. 3, 5.2.2), and
numpy's sort.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libksort_oracle.so")
SOURCES = [os.path.join(_HERE, "ksort_oracle.c")]
CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread"]

_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


class Call(ctypes.Structure):
    """One partition call (Steps 1-4) as the literal steps performed it."""

    _fields_ = [
        ("left", ctypes.c_int64),
        ("right", ctypes.c_int64),
        ("i", ctypes.c_int64),
        ("comparisons", ctypes.c_int64),
        ("k_minus_i", ctypes.c_int64),
        ("key", ctypes.c_double),
        ("temp", ctypes.c_double),
        ("flag", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


def build(out_path: str = LIB_PATH, extra_flags: list[str] | None = None,
          sources: list[str] | None = None) -> str:
    """Compile the oracle with gcc into a shared library; returns its path."""
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), "-o", out_path,
           *(sources or SOURCES), "-I", _HERE]
    subprocess.run(cmd, check=True)
    return out_path


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    for sfx in ("f64", "f32"):
        f = getattr(lib, f"ksort_oracle_partition_{sfx}")
        f.argtypes = [_p, _i64, _i64, ctypes.POINTER(Call)]
        f.restype = _i64
        f = getattr(lib, f"ksort_oracle_sort_{sfx}")
        f.argtypes = [_p, _i64, ctypes.POINTER(_i64), ctypes.POINTER(Call), _i64,
                      ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        f.restype = ctypes.c_int
        f = getattr(lib, f"ksort_oracle_partition_level_{sfx}")
        f.argtypes = [_p, _p, _p, _i64, _p]
        f.restype = ctypes.c_int
        f = getattr(lib, f"ksort_oracle_segmented_{sfx}")
        f.argtypes = [_p, _p, _i64, _p]
        f.restype = ctypes.c_int
        f = getattr(lib, f"ksort_oracle_sort_parallel_{sfx}")
        f.argtypes = [_p, _i64, ctypes.c_int, ctypes.POINTER(_i64)]
        f.restype = ctypes.c_int
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the oracle library (building it first if it is absent)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _sfx(a: np.ndarray) -> str:
    if a.dtype == np.float64:
        return "f64"
    if a.dtype == np.float32:
        return "f32"
    raise TypeError(f"oracle keys must be float64 or float32, got {a.dtype}")


def _check(a: np.ndarray) -> None:
    if a.ndim != 1 or not a.flags.c_contiguous or not a.flags.writeable:
        raise ValueError("oracle arrays must be 1-D, C-contiguous and writeable")


def partition_(a: np.ndarray, left: int, right: int, lib=None) -> tuple[int, dict]:
    """Steps 1-4 on a[left..right] in place; returns (i, call record)."""
    _check(a)
    lib = lib or load()
    rec = Call()
    i = getattr(lib, f"ksort_oracle_partition_{_sfx(a)}")(
        a.ctypes.data, int(left), int(right), ctypes.byref(rec))
    return int(i), rec.as_dict()


def sort_(a: np.ndarray, trace_cap: int = 0, lib=None) -> dict:
    """Steps 1-6 on the whole array in place.

    Returns {"first_pivot", "calls", "comparisons", "trace"}; "trace" holds
    the first ``trace_cap`` call records in call order.
    """
    _check(a)
    lib = lib or load()
    fp, nc, ncmp = _i64(), _i64(), _i64()
    trace = (Call * max(trace_cap, 1))()
    rc = getattr(lib, f"ksort_oracle_sort_{_sfx(a)}")(
        a.ctypes.data, a.size, ctypes.byref(fp), trace, int(trace_cap),
        ctypes.byref(nc), ctypes.byref(ncmp))
    if rc != 0:
        raise MemoryError("oracle stack allocation failed")
    ntr = min(trace_cap, nc.value)
    return {"first_pivot": fp.value, "calls": nc.value, "comparisons": ncmp.value,
            "trace": [trace[t].as_dict() for t in range(ntr)]}


def sort_parallel_(a: np.ndarray, threads: int, lib=None) -> int:
    """Steps 1-6 in place with up to ``threads`` threads (independent
    sub-arrays in parallel, every call literal); returns the first pivot."""
    _check(a)
    lib = lib or load()
    fp = _i64()
    rc = getattr(lib, f"ksort_oracle_sort_parallel_{_sfx(a)}")(a.ctypes.data, a.size, int(threads), ctypes.byref(fp))
    if rc != 0:
        raise MemoryError("oracle allocation or thread start failed")
    return fp.value


def sorted_copy(a: np.ndarray, lib=None) -> tuple[np.ndarray, int]:
    """Returns (K-sorted copy of a, first pivot index)."""
    b = np.array(a, copy=True)
    info = sort_(b, lib=lib)
    return b, info["first_pivot"]


def partition_level_(a: np.ndarray, left: np.ndarray, length: np.ndarray, lib=None) -> np.ndarray:
    """One partition call on each segment, in place; returns the pivot indices."""
    _check(a)
    lib = lib or load()
    left = np.ascontiguousarray(left, dtype=np.int64)
    length = np.ascontiguousarray(length, dtype=np.int64)
    piv = np.empty(left.size, dtype=np.int64)
    rc = getattr(lib, f"ksort_oracle_partition_level_{_sfx(a)}")(
        a.ctypes.data, left.ctypes.data, length.ctypes.data, left.size, piv.ctypes.data)
    if rc != 0:
        raise ValueError("segment with length < 1")
    return piv


def segmented_(a: np.ndarray, offsets: np.ndarray, lib=None) -> np.ndarray:
    """Steps 1-6 on every array of a packed batch, in place; returns the
    first pivot of each array relative to its start."""
    _check(a)
    lib = lib or load()
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = offsets.size - 1
    fps = np.empty(max(nseg, 0), dtype=np.int64)
    rc = getattr(lib, f"ksort_oracle_segmented_{_sfx(a)}")(
        a.ctypes.data, offsets.ctypes.data, nseg, fps.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle stack allocation failed")
    return fps
