"""The seeded input generator: SplitMix64's published outputs, value ranges
and determinism."""
import numpy as np

import synth


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 0: the first three outputs of the reference
    # implementation (Steele, Lea and Flood; also Vigna's splitmix64.c).
    z = synth.splitmix64(0, 0, 3)
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_based_slices_agree():
    a = synth.splitmix64(12345, 0, 1000)
    b = synth.splitmix64(12345, 400, 600)
    assert np.array_equal(a[400:], b)


def test_ranges_and_types():
    f = synth.uniform_f64(1, 100_000)
    assert f.dtype == np.float64 and f.min() >= 0.0 and f.max() < 1.0
    assert not np.signbit(f).any()
    g = synth.uniform_f32(2, 100_000)
    assert g.dtype == np.float32 and g.min() >= 0.0 and g.max() < 1.0
    h = synth.grid16_f64(3, 100_000)
    assert np.array_equal(h * 65536, np.floor(h * 65536))
    assert np.unique(h).size <= 65536
    # means close to 1/2
    assert abs(f.mean() - 0.5) < 0.01 and abs(float(g.mean()) - 0.5) < 0.01


def test_chunked_fill_matches_direct():
    n = (1 << 22) + 17
    a = synth.uniform_f64(9, n)
    z = synth.splitmix64(9, n - 5, 5)
    assert np.array_equal(a[-5:], (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53)


def test_loguniform_bounds():
    v = synth.loguniform_int(9, 4096, 32, 65536)
    assert v.min() >= 32 and v.max() <= 65536
    # log-uniform: about half the mass below the geometric mean
    gm = np.sqrt(32 * 65536)
    assert 0.45 < (v < gm).mean() < 0.55


def test_batched_offsets():
    keys, offs = synth.batched(9, 10, 4096, 32, 65536)
    assert offs[0] == 0 and offs.size == 4097 and np.all(np.diff(offs) >= 32)
    assert keys.size == offs[-1]


def test_serve_stream():
    sizes, is64, t = synth.serve_requests(2000, 12, 13, 11, 1000, 10**7, 0.7, 100.0)
    assert sizes.min() >= 1000 and sizes.max() <= 10**7
    assert 0.65 < is64.mean() < 0.75
    assert np.all(np.diff(t) >= 0) and abs(t[-1] / 2000 - 0.01) < 0.002


def test_torch_twin_matches_numpy():
    import torch
    for seed in (0, 1, 12345, 2**63 + 5):
        a = synth.splitmix64(seed, 10, 5000).view(np.int64)
        b = synth.torch_splitmix64(seed, 10, 5000).numpy()
        assert np.array_equal(a, b)
    for kind, f in (("uniform_f64", synth.uniform_f64), ("uniform_f32", synth.uniform_f32),
                    ("grid16_f64", synth.grid16_f64)):
        x = f(7, 100_003)
        y = synth.torch_fill(kind, 7, 100_003, chunk=30_000).numpy()
        assert x.dtype == y.dtype and np.array_equal(x.view(np.uint8), y.view(np.uint8))
