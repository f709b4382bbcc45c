"""Helpers of the GPU parity tests: device tensors from numpy, oracle
results, and a loud check that the HIP library (not a fallback) is used."""
import sys

import numpy as np

import oracle


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(a: np.ndarray):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t) -> np.ndarray:
    return t.detach().to("cpu").numpy()


def note(msg: str) -> None:
    """Name the case before a GPU step, so a crash log says which one ran."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def oracle_sorted(a: np.ndarray):
    """(K-sorted copy by the literal CPU oracle, first pivot index)."""
    return oracle.sorted_copy(a)


def assert_bit_equal(got: np.ndarray, want: np.ndarray, what: str) -> None:
    assert got.dtype == want.dtype and got.shape == want.shape, what
    if not np.array_equal(got.view(np.uint8), want.view(np.uint8)):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{what}: {bad.size} positions differ, first at {bad[:5]}: "
                             f"got {got[bad[:5]]} want {want[bad[:5]]}")
