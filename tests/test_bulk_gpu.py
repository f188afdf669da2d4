"""GPU parity of the multi-batch insert (bulk build of sec. V-B and its
footnote): n pairs inserted in one call must leave exactly the levels of
ceil(n / b) consecutive insert batches, byte for byte against the cascade
oracle fed those batches one by one, and answer every query as the map
oracle does.  Integer results, tolerance 0."""
import numpy as np
import pytest

from _gpu import Trio, note

pytestmark = pytest.mark.gpu


def pairs(rng, n, domain):
    k = rng.integers(0, domain, n, dtype=np.uint64).astype(np.uint32)
    v = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return k, v


def queries(rng, domain, n=800):
    q = rng.integers(0, domain, n, dtype=np.uint64).astype(np.uint32)
    lo = rng.integers(0, domain, n // 2, dtype=np.uint64).astype(np.uint32)
    hi = np.minimum(lo.astype(np.uint64) + domain // 50 + 1, 2**31 - 1).astype(np.uint32)
    return q, lo, hi


# (b, batches before, pairs in the bulk call, key domain, seed)
CASES = [
    (1, 0, 37, 10, 1),
    (3, 5, 3 * 3, 40, 2),
    (3, 5, 3 * 1, 40, 3),
    (5, 6, 5 * 3 - 2, 100, 4),
    (7, 7, 7 * 3, 1 << 31, 5),
    (64, 0, 64 * 100 + 17, 5000, 6),
    (64, 13, 64 * 51 + 1, 5000, 7),
    (1000, 11, 1000 * 21 + 999, 1 << 31, 8),
    (2048, 0, 2048 * 1027, 1 << 31, 9),   # level 10 of 2^21: digit-pass sort
    (2048, 3, 2048 * 1025, 1 << 20, 10),  # takes over old levels 0 and 1
]


@pytest.mark.parametrize("b,r0,n,domain,seed", CASES)
def test_bulk_insert_equals_sequential_batches(b, r0, n, domain, seed):
    rng = np.random.default_rng(seed)
    note("bulk insert b=%d r0=%d n=%d seed=%d" % (b, r0, n, seed))
    t = Trio(b)
    for i in range(r0):
        k, v = pairs(rng, b if i % 3 else max(1, b // 2), domain)
        if i % 4 == 3:
            t.delete(k)
        else:
            t.insert(k, v)
    k, v = pairs(rng, n, domain)
    t.bulk(k, v)
    t.check_levels()
    t.check_queries(*queries(rng, domain))
    # Ordinary batches and a second bulk call on top.
    k2, v2 = pairs(rng, b, domain)
    t.delete(k2[: max(1, b // 3)])
    k3, v3 = pairs(rng, 3 * b + 1, domain)
    t.bulk(k3, v3)
    t.check_levels()
    t.check_queries(*queries(rng, domain))


def test_bulk_insert_duplicates_inside_the_call():
    """A key repeated across the batches of one call: the last occurrence in
    array order wins, as with sequential batches."""
    b = 256
    note("bulk insert duplicates")
    t = Trio(b)
    keys = np.tile(np.arange(100, dtype=np.uint32), 40)[: 15 * b + 7]
    vals = np.arange(keys.size, dtype=np.uint32)
    t.bulk(keys, vals)
    t.check_levels()
    t.check_queries(np.arange(120, dtype=np.uint32), np.array([0, 50], np.uint32),
                    np.array([99, 200], np.uint32))
