"""lsm_range_async_noalloc (range scratch in the library's fixed array)
against lsm_range_async on the same handle and against the map oracle:
offsets, keys and values bit for bit (integer results, tolerance 0), on two
calls in a row with the second one smaller, so that the fixed array still
holds the first call's counts and look-back words.  Every call is made with
allocation injection set to fail the first allocation, so a call that
allocated anything would return LSM_ENOMEM."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd.lsm import LSM_ECAPACITY, LSM_ENOMEM, LSM_OK
from _gpu import Trio, dev, host, note

pytestmark = pytest.mark.gpu

MAXQ = 1 << 20  # LSM_NOALLOC_MAX_QUERIES


def call(t, name, lo, hi, cap, no_alloc=True):
    """One range call through the C ABI into fresh sentinel-filled outputs;
    returns (status, offsets, keys, vals) on the host."""
    nq = lo.numel()
    offs = torch.full((nq + 1,), -7, dtype=torch.int64, device="cuda")
    keys = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    vals = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    before = t.g.stats().device_bytes
    if no_alloc:
        t.g.fail_alloc_after(0)
    try:
        rc = getattr(t.g._lib, name)(t.g._h, lo.data_ptr(), hi.data_ptr(), nq, offs.data_ptr(),
                                     keys.data_ptr(), vals.data_ptr(), cap)
    finally:
        t.g.fail_alloc_after(-1)
    t.g.sync()
    torch.cuda.synchronize()
    if no_alloc:
        assert t.g.stats().device_bytes == before
    return rc, host(offs), host(keys), host(vals)


def compare(t, lo_np, hi_np, cap=None):
    """Both entry points and the oracle on one query batch."""
    oo, ok, ov = t.m.range(lo_np, hi_np)
    total = int(oo[-1])
    cap = total if cap is None else cap
    lo, hi = dev(lo_np), dev(hi_np)
    note("noalloc range nq=%d total=%d cap=%d levels=%s" % (lo_np.size, total, cap, t.g.occupied()))
    rc_a, oa, ka, va = call(t, "lsm_range_async", lo, hi, cap, no_alloc=False)
    rc_n, on, kn, vn = call(t, "lsm_range_async_noalloc", lo, hi, cap)
    assert rc_a == LSM_OK and rc_n == LSM_OK, (rc_a, rc_n)
    assert np.array_equal(on, oa), "offsets differ from lsm_range_async"
    assert np.array_equal(kn, ka), "keys differ from lsm_range_async"
    assert np.array_equal(vn, va), "values differ from lsm_range_async"
    assert np.array_equal(on, oo), "offsets differ from the oracle"
    # Queries whose pairs end within cap are written, the others not at all.
    fit = int(np.searchsorted(oo[1:], cap, side="right"))
    end = int(oo[fit])
    assert np.array_equal(kn[:end], ok[:end]) and np.array_equal(vn[:end], ov[:end])
    if cap > end:
        assert np.all(kn[end:cap] == np.uint32(0xFFFFFFF9))
    return total


def queries(rng, n, domain, width):
    lo = rng.integers(0, domain, n).astype(np.uint32)
    w = rng.integers(0, width, n).astype(np.uint32)
    hi = (lo + w).astype(np.uint32)
    return lo, hi


def build(b, R, domain, seed, del_every=4):
    rng = np.random.default_rng(seed)
    t = Trio(b)
    for i in range(R):
        k = rng.integers(0, domain, b).astype(np.uint32)
        if i % del_every == del_every - 1:
            t.delete(k)
        else:
            t.insert(k, rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
    return t, rng


@pytest.mark.parametrize("R", [11, 8])  # levels {0, 1, 3} (k-way walk) and one level
def test_noalloc_equals_range_async_twice(R):
    b, domain = 1000, 60000
    t, rng = build(b, R, domain, seed=R)
    # First call at the maximum batch, second smaller: the fixed array keeps
    # the first call's counts and look-back words.
    total = compare(t, *queries(rng, MAXQ, domain, 24))
    assert total > 0
    compare(t, *queries(rng, 1500, domain, 400))
    # A capacity that cuts the output inside the batch.
    lo, hi = queries(rng, 5000, domain, 300)
    full = int(t.m.range(lo, hi)[0][-1])
    compare(t, lo, hi, cap=full // 2)
    t.g.close()


def test_noalloc_settles_staged_elements_and_limits():
    b, domain = 1000, 40000
    t, rng = build(b, 11, domain, seed=5)
    # Staged elements go in first (their level exists: r = 11 -> level 2).
    ks = rng.integers(0, domain, 300).astype(np.uint32)
    vs = rng.integers(0, 2**32, 300, dtype=np.uint64).astype(np.uint32)
    t.g.submit(dev(ks), dev(vs))
    t.m.insert(ks, vs)
    compare(t, *queries(rng, 3000, domain, 200))
    assert t.g.num_batches == 12 and t.g.pending == 0
    # Above the maximum: refused, nothing enqueued.
    lo = dev(np.zeros(MAXQ + 1, np.uint32))
    rc, _, _, _ = call(t, "lsm_range_async_noalloc", lo, lo, 16)
    assert rc == LSM_ECAPACITY
    # No queries: offsets[0] = 0.
    e = dev(np.zeros(0, np.uint32))
    rc, offs, _, _ = call(t, "lsm_range_async_noalloc", e, e, 0)
    assert rc == LSM_OK and offs.tolist() == [0]
    t.g.close()


def test_noalloc_refuses_an_insertion_that_needs_memory():
    b, domain = 512, 30000
    t, rng = build(b, 3, domain, seed=9, del_every=100)  # levels 0, 1; level 2 never reached
    ks = rng.integers(0, domain, 100).astype(np.uint32)
    vs = rng.integers(0, 2**32, 100, dtype=np.uint64).astype(np.uint32)
    t.g.submit(dev(ks), dev(vs))
    lo, hi = queries(rng, 2000, domain, 100)
    rc, _, _, _ = call(t, "lsm_range_async_noalloc", dev(lo), dev(hi), 1 << 16)
    assert rc == LSM_ENOMEM
    assert t.g.num_batches == 3 and t.g.pending == 100
    t.g.flush()  # allocates level 2 and inserts the staged batch
    t.m.insert(ks, vs)
    compare(t, lo, hi)
    t.g.close()
