"""GPU parity with seventeen occupied levels (r = 2^17 - 1 at b = 2).

More than sixteen occupied levels select the widest query instantiations
(32 level slots) of the count pass and of range emission, both from the
count pass's stored cursors and, in the allocation-free range, by searching
again; no smaller dictionary reaches them.  The levels are built by one
bulk insertion (sec. V-B) and 40 single batches of deletions, mixed
operations and insertions over a key domain of 40000, so keys repeat across
many levels with tombstones among them.  Levels byte for byte against the
cascade oracle; lookups, counts, ranges, successors and predecessors
against the map oracle; the allocation-free range equal to lsm_range_async
and to the oracle.  Integer results, tolerance 0."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd.lsm import LSM_OK
from _gpu import Trio, dev, host, note

pytestmark = pytest.mark.gpu


def range_call(t, name, lo, hi, cap):
    nq = lo.numel()
    offs = torch.full((nq + 1,), -7, dtype=torch.int64, device="cuda")
    keys = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    vals = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = getattr(t.g._lib, name)(t.g._h, lo.data_ptr(), hi.data_ptr(), nq, offs.data_ptr(),
                                 keys.data_ptr(), vals.data_ptr(), cap)
    t.g.sync()
    torch.cuda.synchronize()
    return rc, host(offs), host(keys), host(vals)


def test_seventeen_levels_take_the_widest_walks():
    b, domain, tail = 2, 40000, 40
    R = (1 << 17) - 1
    rng = np.random.default_rng(1717)
    t = Trio(b)
    n0 = b * (R - tail)
    note("seventeen levels: bulk %d pairs at b=%d, then %d batches" % (n0, b, tail))
    k = rng.integers(0, domain, n0, dtype=np.uint64).astype(np.uint32)
    v = rng.integers(0, 2**32, n0, dtype=np.uint64).astype(np.uint32)
    t.bulk(k, v)
    for i in range(tail):
        kk = rng.integers(0, domain, b, dtype=np.uint64).astype(np.uint32)
        vv = rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32)
        if i % 3 == 0:
            t.delete(kk)
        elif i % 3 == 1:
            t.mixed(kk, vv, np.array([1, 0], np.uint8))
        else:
            t.insert(kk, vv)
    assert t.g.num_batches == R and len(t.g.occupied()) == 17
    t.check_levels()
    q = rng.integers(0, domain + 10, 4000, dtype=np.uint64).astype(np.uint32)
    lo = rng.integers(0, domain, 2000, dtype=np.uint64).astype(np.uint32)
    hi = (lo.astype(np.uint64) + rng.integers(0, 400, lo.size)).astype(np.uint32)
    lo[:7] = np.maximum(lo[:7], 1)
    hi[:7] = lo[:7] - 1  # empty ranges (lo > hi)
    note("seventeen levels: queries")
    t.check_queries(q, lo, hi)
    t.check_order(q)
    oo, ok, ov = t.m.range(lo, hi)
    total = int(oo[-1])
    rc_a, oa, ka, va = range_call(t, "lsm_range_async", dev(lo), dev(hi), total)
    rc_n, on, kn, vn = range_call(t, "lsm_range_async_noalloc", dev(lo), dev(hi), total)
    assert rc_a == LSM_OK and rc_n == LSM_OK, (rc_a, rc_n)
    assert np.array_equal(oa, oo) and np.array_equal(on, oo), "range offsets differ"
    assert np.array_equal(ka[:total], ok) and np.array_equal(kn[:total], ok), "range keys differ"
    assert np.array_equal(va[:total], ov) and np.array_equal(vn[:total], ov), "range values differ"
    t.g.close()
