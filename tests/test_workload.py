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
