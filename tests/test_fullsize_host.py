"""CPU checks of the host helpers the full-size parity tests rely on, and of
the key classes the query recipe draws hits and misses from."""
import numpy as np

import oracle
from paper_1707_05354_amd import workload as W
from _fullsize import FilteredMap, key_filter, ops_touching


def test_ops_touching_equals_a_direct_key_test():
    rng = np.random.default_rng(5)
    for domain in (50, 1 << 20, 1 << 31):
        keys = rng.integers(0, domain, 20000).astype(np.uint32)
        pts = rng.integers(0, domain, 40).astype(np.uint32)
        lo = rng.integers(0, domain, 30).astype(np.uint32)
        hi = np.minimum(lo.astype(np.int64) + rng.integers(0, max(2, domain // 100), 30),
                        domain - 1).astype(np.uint32)
        hi[:3] = lo[:3]  # one-key intervals
        if lo.size > 5:
            lo[4], hi[4] = hi[4], lo[4]  # an empty (reversed) interval selects nothing
        want = np.flatnonzero(key_filter(pts, lo[hi >= lo], hi[hi >= lo])(keys))
        got = ops_touching(keys, pts, lo[hi >= lo], hi[hi >= lo])
        assert np.array_equal(got, want), domain


def test_filtered_map_answers_like_the_full_map():
    rng = np.random.default_rng(6)
    full, ops = oracle.MapOracle(), []
    for t in range(30):
        k = rng.integers(0, 500, 64).astype(np.uint32)
        v = rng.integers(0, 2**32, 64, dtype=np.uint64).astype(np.uint32)
        d = (rng.random(64) < 0.3).astype(np.uint8)
        ops.append((k, v, d))
    q = rng.integers(0, 500, 50).astype(np.uint32)
    lo = rng.integers(0, 480, 10).astype(np.uint32)
    hi = lo + 15
    fm = FilteredMap(key_filter(q, lo, hi))
    for k, v, d in ops:
        fm.mixed_in_order(k, v, d)
        for j in range(k.size):  # one operation at a time
            if d[j]:
                full.delete(k[j:j + 1])
            else:
                full.insert(k[j:j + 1], v[j:j + 1])
    assert all(np.array_equal(a, b) for a, b in zip(fm.m.lookup(q), full.lookup(q)))
    assert np.array_equal(fm.m.count(lo, hi), full.count(lo, hi))
    assert all(np.array_equal(a, b) for a, b in zip(fm.m.range(lo, hi), full.range(lo, hi)))


def test_key_classes_agree_with_the_dictionary():
    """Keys the recipe calls sure-present are present at the end, keys it
    calls sure-absent are absent, and every inserted key is listed."""
    rng = np.random.default_rng(7)
    for t in range(5):
        R, b = 30, 40
        keys = rng.integers(0, 300, (R, b)).astype(np.uint32)
        vals = rng.integers(0, 2**32, (R, b), dtype=np.uint64).astype(np.uint32)
        is_delete = rng.random(R) < 0.3
        is_delete[0] = False
        m = oracle.MapOracle()
        for i in range(R):
            (m.delete(keys[i]) if is_delete[i] else m.insert(keys[i], vals[i]))
        live, dead, inserted = W._key_classes(keys.reshape(-1), np.repeat(np.arange(R), b),
                                              np.repeat(is_delete, b))
        assert np.all(m.lookup(live)[1] == 1)
        assert np.all(m.lookup(dead)[1] == 0)
        assert np.array_equal(inserted, np.unique(keys[~is_delete]))


def test_tiny_query_recipe_hits_half():
    w = W.tiny()
    m = oracle.MapOracle()
    for i in range(w.R):
        (m.delete(w.keys[i]) if w.is_delete[i] else m.insert(w.keys[i], w.vals[i]))
    f = m.lookup(w.lookups)[1]
    hit = (W.splitmix64(1, 4, 0, w.lookups.size) & np.uint64(1)).astype(bool)
    assert np.all(f[hit] == 1) and np.all(f[~hit] == 0)
    assert 7.0 < m.count(w.count_lo, w.count_hi).mean() < 9.5
