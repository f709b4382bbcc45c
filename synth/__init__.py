"""Seeded synthetic inputs for K-sort workloads (numpy).

This module draws inputs only; it holds none of the sorting method's
arithmetic, and both the HIP library's tests and the CPU oracle's tests take
their inputs from it.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used as a counter-based generator.  Element
t of stream `seed` is the SplitMix64 output mixing function applied to the
state seed + (t + 1) * 0x9E3779B97F4A7C15 (mod 2^64):

    z = state
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

Derived variates (the paper's workload is i.i.d. continuous U[0,1],
arXiv 1107.3622 Section 2):
    f64 U[0,1)         (z >> 11) * 2^-53
    f32 U[0,1)         (z >> 40) * 2^-24
    2^16-value grid    (z >> 48) * 2^-16            (heavy duplicates)
    log-uniform int    floor(exp(ln a + u * (ln b - ln a))), u the f64 variate,
                       clamped to [a, b]

None of these can produce NaN or -0.0.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

_CHUNK = 1 << 22


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Raw 64-bit outputs for element indices start .. start+count-1."""
    with np.errstate(over="ignore"):
        t = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + t * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def _fill(seed: int, n: int, dtype, conv) -> np.ndarray:
    out = np.empty(n, dtype=dtype)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        out[s:s + c] = conv(splitmix64(seed, s, c))
    return out


def uniform_f64(seed: int, n: int) -> np.ndarray:
    """n i.i.d. U[0,1) doubles with 53 random bits."""
    return _fill(seed, n, np.float64,
                 lambda z: (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53))


def uniform_f32(seed: int, n: int) -> np.ndarray:
    """n i.i.d. U[0,1) floats with 24 random bits."""
    return _fill(seed, n, np.float32,
                 lambda z: ((z >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)).astype(np.float32))


def grid16_f64(seed: int, n: int) -> np.ndarray:
    """n doubles drawn uniformly from the 2^16-value grid {k / 2^16}."""
    return _fill(seed, n, np.float64,
                 lambda z: (z >> np.uint64(48)).astype(np.float64) * (2.0 ** -16))


def loguniform_int(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count integers, log-uniform in [lo, hi]."""
    u = uniform_f64(seed, count)
    la, lb = math.log(lo), math.log(hi)
    v = np.floor(np.exp(la + u * (lb - la))).astype(np.int64)
    return np.clip(v, lo, hi)


def batched(len_seed: int, data_seed: int, nseg: int, lo: int, hi: int,
            dtype=np.float64) -> tuple[np.ndarray, np.ndarray]:
    """A packed batch: nseg arrays with log-uniform lengths in [lo, hi]
    (stream len_seed) and U[0,1) keys over the packed buffer (stream
    data_seed).  Returns (keys, offsets[nseg + 1])."""
    lens = loguniform_int(len_seed, nseg, lo, hi)
    offsets = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    n = int(offsets[-1])
    keys = uniform_f64(data_seed, n) if dtype == np.float64 else uniform_f32(data_seed, n)
    return keys, offsets


def serve_requests(count: int, size_seed: int, dtype_seed: int, arrival_seed: int,
                   lo: int, hi: int, p_f64: float, rate_per_s: float):
    """A seeded request stream: sizes log-uniform in [lo, hi], dtype f64 with
    probability p_f64, Poisson arrivals at rate_per_s (exponential gaps).
    Returns (sizes int64, is_f64 bool, arrival times in seconds).  Request r's
    keys come from stream 1_000_000 + r."""
    sizes = loguniform_int(size_seed, count, lo, hi)
    is_f64 = uniform_f64(dtype_seed, count) < p_f64
    u = uniform_f64(arrival_seed, count)
    gaps = -np.log1p(-u) / rate_per_s
    return sizes, is_f64, np.cumsum(gaps)


REQUEST_SEED_BASE = 1_000_000


# ---------------------------------------------------------------- torch twin
# The same counter-based generator written with torch int64 arithmetic, so
# large inputs can be drawn directly in device memory.  int64 products wrap
# modulo 2^64 exactly like the uint64 ones above; right shifts are made
# logical by masking.  test_synth checks it bit for bit against numpy.

def _to_i64(c: int) -> int:
    return c - (1 << 64) if c >= (1 << 63) else c


_G64, _M164, _M264 = _to_i64(0x9E3779B97F4A7C15), _to_i64(0xBF58476D1CE4E5B9), _to_i64(0x94D049BB133111EB)


def _srl(z, k: int):
    return (z >> k) & ((1 << (64 - k)) - 1)


def torch_splitmix64(seed: int, start: int, count: int, device="cpu"):
    import torch
    t = torch.arange(start + 1, start + 1 + count, dtype=torch.int64, device=device)
    z = t * _G64 + _to_i64(seed & 0xFFFFFFFFFFFFFFFF)
    z = (z ^ _srl(z, 30)) * _M164
    z = (z ^ _srl(z, 27)) * _M264
    return z ^ _srl(z, 31)


def torch_fill(kind: str, seed: int, n: int, device="cpu", chunk: int = 1 << 26):
    """Device-resident twin of uniform_f64 / uniform_f32 / grid16_f64."""
    import torch
    dt = torch.float32 if kind == "uniform_f32" else torch.float64
    out = torch.empty(n, dtype=dt, device=device)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        z = torch_splitmix64(seed, s, c, device)
        if kind == "uniform_f64":
            out[s:s + c] = _srl(z, 11).to(torch.float64) * (2.0 ** -53)
        elif kind == "uniform_f32":
            out[s:s + c] = (_srl(z, 40).to(torch.float64) * (2.0 ** -24)).to(torch.float32)
        elif kind == "grid16_f64":
            out[s:s + c] = _srl(z, 48).to(torch.float64) * (2.0 ** -16)
        else:
            raise ValueError(kind)
        del z
    return out


def torch_make(name: str, device="cpu"):
    w = WORKLOADS[name]
    return torch_fill(w["kind"], w["seed"], w["n"], device)

# Named workloads: (description, seed) in the shapes the benchmark and the
# parity tests use.
WORKLOADS = {
    "c0_n1e5_f64": dict(kind="uniform_f64", n=100_000, seed=1),
    "c1_n1e6_f64": dict(kind="uniform_f64", n=1_000_000, seed=2),
    "c1_n2.5e6_f64": dict(kind="uniform_f64", n=2_500_000, seed=3),
    "c1_n7e6_f64": dict(kind="uniform_f64", n=7_000_000, seed=4),
    "c1_n1e7_f64": dict(kind="uniform_f64", n=10_000_000, seed=5),
    "c2_n2^28_f64": dict(kind="uniform_f64", n=1 << 28, seed=6),
    "c2_n2^29_f32": dict(kind="uniform_f32", n=1 << 29, seed=7),
    "c2_grid16_n1e7_f64": dict(kind="grid16_f64", n=10_000_000, seed=8),
}


def make(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    return {"uniform_f64": uniform_f64, "uniform_f32": uniform_f32,
            "grid16_f64": grid16_f64}[w["kind"]](w["seed"], w["n"])
