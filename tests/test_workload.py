"""The seeded generator: determinism, counter-based slicing, recipe shapes."""
import numpy as np

from paper_1707_05354_amd import workload as W


def test_splitmix64_reference_values():
    # splitmix64 with state 0: the first outputs of the published generator.
    z = W.splitmix64(0, 0, 0, 3)
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_based_slices_agree():
    a = W.splitmix64(3, 1, 0, 1000)
    b = W.splitmix64(3, 1, 400, 100)
    assert np.array_equal(a[400:500], b)


def test_tiny_recipe():
    w = W.tiny()
    assert w.keys.shape == (20, 1024) and w.keys.dtype == np.uint32
    assert int(w.keys.max()) < 2**31
    assert w.is_delete.tolist() == [False] * 16 + [True] * 4
    ins = set(w.keys[:16].reshape(-1).tolist())
    assert set(w.keys[16:].reshape(-1).tolist()) <= ins
    assert w.lookups.size == 4096 and w.count_lo.size == 1024 and w.range_lo.size == 1024
    assert np.all(w.count_hi >= w.count_lo) and int(w.count_hi.max()) < 2**31
    w2 = W.tiny()
    assert np.array_equal(w.keys, w2.keys) and np.array_equal(w.lookups, w2.lookups)


def test_paper_scale_shape_small_variant():
    w = W.paper_scale(b=256, R=40, nq=1000, ncount=100)
    assert w.keys.shape == (40, 256)
    assert w.is_delete.sum() == 4 and w.is_delete[9] and w.is_delete[39]


def test_zipf_keys_law_and_bijection():
    """Zipf(1.1) ranks: frequencies of the first ranks follow k^-1.1 and the
    rank-to-key map is a bijection of [0, 2^24)."""
    r = W.zipf_ranks(9, 7, 0, 1 << 20)
    c = np.bincount(r, minlength=8)
    ratio = c[1] / c[2]
    assert abs(ratio - 2 ** 1.1) < 0.05
    assert r.min() >= 1 and r.max() <= 1 << 24
    k = W.zipf_keys(9, 7, 0, 1 << 16)
    assert int(k.max()) < 1 << 24
    # bijection: distinct ranks give distinct keys
    rr = W.zipf_ranks(9, 7, 0, 1 << 16)
    assert np.unique(rr).size == np.unique(k).size


def test_zipf_sweep_points_share_the_key_stream():
    a = W.zipf_sweep(1 << 13, n_total=1 << 18, nq=1 << 10)
    b = W.zipf_sweep(1 << 15, n_total=1 << 18, nq=1 << 10)
    assert np.array_equal(a.keys.reshape(-1), b.keys.reshape(-1))
    assert a.R == 32 and b.R == 8 and a.is_delete.sum() == 6 and b.is_delete.sum() == 1
