"""GPU parity of cleanup (sec. III-E, IV-D) and of the order queries of the
sec. I-B footnote.  Integer results, tolerance 0: after a cleanup every
level must equal the cascade oracle's cleanup byte for byte (placebos
included), and every lookup / count / range / successor / predecessor
answer must equal the map oracle's, before and after the cleanup and after
further batches on top of it."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd import workload as W
from _gpu import Trio, dev, host, note

pytestmark = pytest.mark.gpu

TOP = 2**31 - 1


def order_queries(rng, t, domain, n=600):
    live, _ = t.m.items()
    parts = [rng.integers(0, min(domain + 2, 2**32), n, dtype=np.uint64),
             np.array([0, 1, TOP - 1, TOP, TOP + 1, 2**32 - 1], np.uint64)]
    if live.size:
        pick = live[rng.integers(0, live.size, n // 2)].astype(np.uint64)
        parts += [pick, pick + 1, np.maximum(pick, 1) - 1]
    return np.concatenate(parts).astype(np.uint32)


def apply(t, ops):
    for kind, k, v in ops:
        if kind == "insert":
            t.insert(k, v)
        else:
            t.delete(k)


CASES = [
    # (b, key domain, batches, seed)
    (1, 8, 40, 11),
    (3, 40, 23, 12),
    (7, 1 << 31, 19, 13),
    (64, 300, 31, 14),
    (2047, 4000, 11, 15),
    (2049, 1 << 31, 9, 16),
    (4096, 1 << 15, 37, 17),
]


@pytest.mark.parametrize("b,domain,R,seed", CASES)
def test_order_queries(b, domain, R, seed):
    """Successor / predecessor over several occupied levels holding stale
    elements and tombstones."""
    ops, _q, _lo, _hi = W.random_small(seed, b, R, domain, p_delete=0.3, nq=10)
    note("order queries b=%d domain=%d R=%d seed=%d" % (b, domain, R, seed))
    t = Trio(b)
    rng = np.random.default_rng(seed)
    for j, op in enumerate(ops):
        apply(t, [op])
        if j % 5 == 4 or j == len(ops) - 1:
            t.check_order(order_queries(rng, t, domain))


@pytest.mark.parametrize("b,domain,R,seed", CASES)
def test_cleanup_layout_and_answers(b, domain, R, seed):
    ops, q, lo, hi = W.random_small(seed, b, R, domain, p_delete=0.3, nq=500)
    note("cleanup b=%d domain=%d R=%d seed=%d" % (b, domain, R, seed))
    t = Trio(b)
    apply(t, ops)
    t.check_levels()
    t.cleanup()
    t.check_levels()
    t.check_queries(q, lo, hi)
    rng = np.random.default_rng(seed + 100)
    t.check_order(order_queries(rng, t, domain))
    # Batches on top of the cleaned structure, then a second cleanup.
    more, q2, lo2, hi2 = W.random_small(seed + 1000, b, 9, domain, p_delete=0.3, nq=500)
    for op in more:
        apply(t, [op])
        t.check_levels()
    t.check_queries(q2, lo2, hi2)
    t.check_order(order_queries(rng, t, domain))
    t.cleanup()
    t.check_levels()
    t.check_queries(q2, lo2, hi2)
    t.g.close()


def test_cleanup_many_tiles_and_levels():
    """r = 37 batches of b = 4096 (levels 0, 2, 5): 74 compaction tiles, with
    the new levels' boundaries falling inside tiles."""
    b, R = 4096, 37
    rng = np.random.default_rng(77)
    note("cleanup many tiles b=%d R=%d" % (b, R))
    t = Trio(b)
    for i in range(R):
        k = rng.integers(0, 1 << 17, b).astype(np.uint32)
        if i % 4 == 3:
            t.delete(k[: b // 2])
        else:
            t.insert(k, rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
    assert t.g.occupied() == [0, 2, 5]
    v = t.cleanup()
    assert 0 < v < R * b
    t.check_levels()
    t.check_order(order_queries(rng, t, 1 << 17, n=4000))
    lo = rng.integers(0, 1 << 17, 2000).astype(np.uint32)
    t.check_queries(lo, lo, (lo + 40).astype(np.uint32))


def test_cleanup_special_cases():
    b = 1000
    note("cleanup special cases")
    t = Trio(b)
    assert t.cleanup() == 0 and t.g.num_batches == 0
    keys = np.arange(0, 5000, 3, dtype=np.uint32)
    t.insert(keys[:b], keys[:b] + 1)
    t.insert(keys[b:], keys[b:] + 1)
    t.delete(keys[:b])
    t.delete(keys[b:])
    assert t.cleanup() == 0 and t.g.num_batches == 0 and t.g.occupied() == []
    t.check_order(np.array([0, 5, 4999, TOP], np.uint32))
    # A live key 2^31 - 1 next to the placebos of its own key.
    t.insert(np.array([TOP, 17, 4], np.uint32), np.array([5, 6, 7], np.uint32))
    assert t.cleanup() == 3
    t.check_levels()
    kv, _v = t.g.level(0)
    assert host(kv)[3:].tolist() == [0xFFFFFFFE] * (b - 3)
    t.check_queries(np.array([TOP, 17, 4, 5], np.uint32), np.array([0, TOP], np.uint32),
                    np.array([TOP, TOP], np.uint32))
    t.check_order(np.array([0, 4, 17, TOP - 1, TOP, 2**32 - 1], np.uint32))
    # Exactly b valid pairs: no placebo at all; cleanup twice is the identity.
    t2 = Trio(b)
    t2.insert(np.arange(b, dtype=np.uint32) * 2, np.arange(b, dtype=np.uint32))
    t2.insert(np.arange(b, dtype=np.uint32) * 2 + 1, np.arange(b, dtype=np.uint32))
    t2.delete(np.arange(b, dtype=np.uint32) * 2)
    assert t2.cleanup() == b and t2.g.num_batches == 1
    t2.check_levels()
    before = host(t2.g.level(0)[0]).copy()
    assert t2.cleanup() == b
    t2.check_levels()
    assert np.array_equal(host(t2.g.level(0)[0]), before)
