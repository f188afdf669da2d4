"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer results, so the bar is bit-exactness: every occupied level (key
variables and values, stale elements and tombstones included) must equal
the cascade oracle byte for byte, r and the merge count must match, and
every lookup / count / range answer must equal the map oracle's.
"""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import LSM, LSMError, LSM_EBATCH, LSM_ECAPACITY, LSM_EKEY
from _gpu import Trio, dev, dev_u8, host, note

pytestmark = pytest.mark.gpu


def test_tiny_workload_b1024():
    """b = 1024, 16 insert + 4 delete batches, 4096 lookups, 1024 count and
    1024 range queries (about 8 hits each)."""
    w = W.tiny()
    note("tiny b=1024")
    t = Trio(w.b)
    for i in range(w.R):
        if w.is_delete[i]:
            t.delete(w.keys[i])
        else:
            t.insert(w.keys[i], w.vals[i])
        t.check_levels()
    assert t.g.occupied() == [2, 4]
    t.check_queries(w.lookups, w.count_lo, w.count_hi)
    t.check_queries(w.lookups[:10], w.range_lo, w.range_hi)
    assert 4 <= float(host(t.g.count(dev(w.count_lo), dev(w.count_hi))).mean()) <= 12


CASES = [
    # (b, key domain, batches, seed)
    (1, 8, 40, 1),
    (2, 16, 33, 2),
    (3, 1 << 31, 20, 3),
    (7, 50, 37, 4),
    (64, 200, 31, 5),
    (2047, 3000, 9, 6),
    (2048, 1 << 31, 9, 7),
    (2049, 5000, 9, 8),
    (6161, 1 << 20, 7, 9),
]


@pytest.mark.parametrize("b,domain,R,seed", CASES)
def test_random_streams(b, domain, R, seed):
    """Partial batches (padding), duplicates inside and across batches,
    deletes of present and absent keys, b across sort/merge tile edges."""
    ops, q, lo, hi = W.random_small(seed, b, R, domain, p_delete=0.3, nq=700)
    note("random stream b=%d domain=%d R=%d seed=%d" % (b, domain, R, seed))
    t = Trio(b)
    for j, (kind, k, v) in enumerate(ops):
        if kind == "insert":
            t.insert(k, v)
        else:
            t.delete(k)
        t.check_levels()
        if j % 5 == 4:
            t.check_queries(q, lo, hi)
    t.check_queries(q, lo, hi)


@pytest.mark.parametrize("b", [1, 5, 300, 4096])
def test_mixed_batches(b):
    """Insertions and deletions in one batch; a key inserted and deleted in
    the same batch is deleted (sec. III-A rule 5)."""
    rng = np.random.default_rng(b)
    note("mixed b=%d" % b)
    t = Trio(b)
    for _ in range(13):
        n = int(rng.integers(1, b + 1))
        k = rng.integers(0, max(4, b // 2), n).astype(np.uint32)
        v = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        d = (rng.random(n) < 0.35).astype(np.uint8)
        t.mixed(k, v, d)
        t.check_levels()
    dom = max(4, b // 2) + 2
    q = np.arange(dom, dtype=np.uint32)
    t.check_queries(q, q[: dom // 2], q[dom // 2:dom // 2 * 2])


def test_many_levels_b1():
    """b = 1 and 4095 batches: twelve occupied levels at once."""
    rng = np.random.default_rng(12)
    note("b=1 R=4095")
    t = Trio(1)
    keys = rng.integers(0, 3000, 4095).astype(np.uint32)
    vals = rng.integers(0, 2**32, 4095, dtype=np.uint64).astype(np.uint32)
    dels = rng.random(4095) < 0.2
    for i in range(4095):
        if dels[i]:
            t.delete(keys[i:i + 1])
        else:
            t.insert(keys[i:i + 1], vals[i:i + 1])
    assert len(t.g.occupied()) == 12
    t.check_levels()
    q = np.arange(3002, dtype=np.uint32)
    lo = rng.integers(0, 3002, 2000).astype(np.uint32)
    hi = np.minimum(lo + rng.integers(0, 300, 2000), 3001).astype(np.uint32)
    t.check_queries(q, lo, hi)


def test_large_batches_many_tiles():
    """b = 2^19 + 3: 257 sort tiles with a ragged tail, then merges of
    2^19 + 3 runs spanning hundreds of merge tiles; heavy duplication."""
    b = (1 << 19) + 3
    rng = np.random.default_rng(19)
    note("b=2^19+3")
    t = Trio(b)
    for r in range(3):
        k = rng.integers(0, 1 << 18, b).astype(np.uint32)
        v = rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32)
        t.insert(k, v)
        t.check_levels()
    t.delete(rng.integers(0, 1 << 18, b // 3).astype(np.uint32))
    t.check_levels()
    q = rng.integers(0, (1 << 18) + 5, 20000).astype(np.uint32)
    lo = rng.integers(0, 1 << 18, 5000).astype(np.uint32)
    t.check_queries(q, lo, lo + 40)


def test_all_equal_keys_and_extremes():
    """Every key equal (one long run through every merge tile), then keys 0
    and 2^31-1 with values 0 and 2^32-1, and bounds up to 2^32-1."""
    b = 5000
    note("all-equal keys b=5000")
    t = Trio(b)
    for r in range(4):
        t.insert(np.full(b, 77, np.uint32), np.arange(r * b, (r + 1) * b, dtype=np.uint32))
        t.check_levels()
    t.insert(np.array([0, 2**31 - 1, 77], np.uint32), np.array([0, 2**32 - 1, 5], np.uint32))
    t.check_levels()
    t.delete(np.array([77], np.uint32))
    t.check_levels()
    q = np.array([0, 1, 76, 77, 78, 2**31 - 2, 2**31 - 1, 2**31, 2**32 - 1], np.uint32)
    lo = np.array([0, 0, 77, 78, 2**31 - 1, 5, 0], np.uint32)
    hi = np.array([2**32 - 1, 2**31 - 1, 77, 2**31 - 1, 2**31 - 1, 4, 0], np.uint32)
    t.check_queries(q, lo, hi)


def test_empty_dictionary_and_empty_queries():
    note("empty dictionary")
    g = LSM(256)
    q = dev(np.array([0, 5, 2**31 - 1], np.uint32))
    v, f = g.lookup(q)
    assert host(f).tolist() == [0, 0, 0] and host(v).tolist() == [0, 0, 0]
    assert host(g.count(q, q)).tolist() == [0, 0, 0]
    off, k, val = g.range(q, q)
    assert host(off).tolist() == [0, 0, 0, 0] and k.numel() == 0
    e = dev(np.zeros(0, np.uint32))
    v, f = g.lookup(e)
    assert v.numel() == 0
    assert g.count(e, e).numel() == 0
    off, k, val = g.range(e, e)
    assert host(off).tolist() == [0]
    g.insert(e, e)  # n == 0: no-op
    assert g.num_batches == 0
    g.close()


def test_batch_size_errors_leave_state_unchanged():
    note("batch size errors")
    t = Trio(8)
    t.insert(np.arange(8, dtype=np.uint32), np.arange(8, dtype=np.uint32))
    with pytest.raises(LSMError) as ei:
        t.g.insert(dev(np.arange(9, dtype=np.uint32)), dev(np.arange(9, dtype=np.uint32)))
    assert ei.value.status == LSM_EBATCH
    with pytest.raises(LSMError):
        t.g.delete(dev(np.arange(9, dtype=np.uint32)))
    t.check_levels()


@pytest.mark.parametrize("key_bits", [31, 24])
def test_checked_mode_rejects_out_of_range_keys(key_bits):
    note("checked mode key_bits=%d" % key_bits)
    t = Trio(16, key_bits=key_bits, checked=True)
    rng = np.random.default_rng(key_bits)
    for _ in range(3):
        t.insert(rng.integers(0, 1 << key_bits, 16).astype(np.uint32),
                 rng.integers(0, 2**32, 16, dtype=np.uint64).astype(np.uint32))
    before = t.g.num_batches
    bad = rng.integers(0, 1 << key_bits, 16).astype(np.uint32)
    bad[7] = 1 << key_bits
    with pytest.raises(LSMError) as ei:
        t.g.insert(dev(bad), dev(bad))
    assert ei.value.status == LSM_EKEY
    with pytest.raises(LSMError):
        t.g.delete(dev(bad))
    assert t.g.num_batches == before
    t.check_levels()
    t.insert(bad[:7], bad[:7])
    t.check_levels()


def test_key_bits_24_fewer_passes():
    """Keys < 2^24 sorted with three digit passes give the same layout."""
    rng = np.random.default_rng(24)
    note("key_bits=24 b=8192")
    t = Trio(8192, key_bits=24)
    for r in range(6):
        k = rng.integers(0, 1 << 24, 8192).astype(np.uint32)
        if r % 3 == 2:
            t.delete(k[:4000])
        else:
            t.insert(k, rng.integers(0, 2**32, 8192, dtype=np.uint64).astype(np.uint32))
        t.check_levels()
    q = rng.integers(0, 1 << 24, 4000).astype(np.uint32)
    t.check_queries(q, q, q + 5000)


def test_range_two_phase_capacity():
    note("range capacity")
    t = Trio(1024)
    rng = np.random.default_rng(3)
    for _ in range(3):
        t.insert(rng.integers(0, 10000, 1024).astype(np.uint32),
                 rng.integers(0, 2**32, 1024, dtype=np.uint64).astype(np.uint32))
    lo = dev(np.array([0, 100, 5000], np.uint32))
    hi = dev(np.array([50, 3000, 9999], np.uint32))
    off = torch.empty(4, dtype=torch.int64, device="cuda")
    with pytest.raises(LSMError) as ei:
        t.g.range_raw(lo, hi, off, None, None, 0)
    assert ei.value.status == LSM_ECAPACITY
    want_off, want_k, want_v = t.m.range(np.array([0, 100, 5000]), np.array([50, 3000, 9999]))
    torch.cuda.synchronize()
    assert np.array_equal(host(off), want_off)
    k = torch.empty(int(want_off[-1]), dtype=torch.int32, device="cuda")
    v = torch.empty(int(want_off[-1]), dtype=torch.int32, device="cuda")
    assert t.g.range_raw(lo, hi, off, k, v, int(want_off[-1])) == int(want_off[-1])
    torch.cuda.synchronize()
    assert np.array_equal(host(k), want_k) and np.array_equal(host(v), want_v)


def test_one_level_ranges_over_long_runs():
    """Ranges over one occupied level (emitted one query at a time per wave,
    64 candidates a chunk): key runs far longer than a chunk (batches of one
    key, the padding of partial batches), a tombstone run under newer
    insertions of the same key, ranges starting and ending inside runs, the
    whole key space, and a capacity that cuts the output."""
    b = 3000
    note("one-level ranges over long runs b=%d" % b)
    rng = np.random.default_rng(21)
    t = Trio(b)

    def vals(n):
        return rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)

    t.insert(np.full(b, 500, np.uint32), vals(b))
    t.insert(rng.integers(0, 2000, 37).astype(np.uint32), vals(37))  # 2963 padding copies
    t.delete(np.full(b, 700, np.uint32))
    t.insert(np.full(b, 700, np.uint32), vals(b))
    t.mixed(rng.integers(0, 2000, b).astype(np.uint32), vals(b),
            (rng.random(b) < 0.5).astype(np.uint8))
    t.insert(rng.integers(0, 2000, b).astype(np.uint32), vals(b))
    t.delete(rng.integers(0, 2000, 500).astype(np.uint32))
    t.insert(np.full(b, 500, np.uint32), vals(b))
    t.check_levels()
    assert t.g.occupied() == [3]
    lo = np.r_[np.array([500, 499, 0, 700, 699, 701, 0, 2000], np.uint32),
               rng.integers(0, 2100, 3000).astype(np.uint32)]
    hi = np.r_[np.array([500, 501, 2**31 - 1, 700, 700, 2**32 - 1, 499, 1999], np.uint32),
               (lo[8:] + rng.integers(0, 300, 3000)).astype(np.uint32)]
    q = np.arange(0, 2100, dtype=np.uint32)
    t.check_queries(q, lo, hi)
    # A capacity inside the output: lsm_range writes nothing and reports the
    # total; lsm_range_async writes the queries that fit, in full.
    want_off, want_k, want_v = t.m.range(lo, hi)
    cap = int(want_off[-1]) // 2
    off = torch.empty(lo.size + 1, dtype=torch.int64, device="cuda")
    k = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    v = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(LSMError) as ei:
        t.g.range_raw(dev(lo), dev(hi), off, k, v, cap)
    assert ei.value.status == LSM_ECAPACITY
    torch.cuda.synchronize()
    assert np.array_equal(host(off), want_off) and np.all(host(k) == np.uint32(0xFFFFFFFF))
    t.g.range_async(dev(lo), dev(hi), off, k, v, cap)
    torch.cuda.synchronize()
    end = int(want_off[np.searchsorted(want_off[1:], cap, side="right")])
    assert np.array_equal(host(off), want_off)
    assert np.array_equal(host(k)[:end], want_k[:end]) and np.array_equal(host(v)[:end], want_v[:end])
    assert np.all(host(k)[end:] == np.uint32(0xFFFFFFFF))
    t.g.close()


def test_merges_with_several_tiles_per_workgroup():
    """b = 2^20 + 5: merges of 2^21 + 10 and 2^22 + 20 outputs need more
    tiles than work-groups, so each work-group walks a run of tiles (ragged
    last run), and one key is hot enough to span many tiles."""
    b = (1 << 20) + 5
    rng = np.random.default_rng(20)
    note("b=2^20+5 multi-tile merges")
    t = Trio(b)
    for r in range(4):
        k = rng.integers(0, 1 << 30, b).astype(np.uint32)
        k[rng.random(b) < 0.05] = 12345
        t.insert(k, rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
        t.check_levels()
    q = np.concatenate([np.array([12345], np.uint32), rng.integers(0, 1 << 30, 5000).astype(np.uint32)])
    t.check_queries(q, q[:2000], q[:2000] + 200000)


def test_one_oversized_sort_bucket():
    """Keys below 2^16 share one top digit, so the batch sort's whole batch
    (98311 elements, beyond what one work-group sorts in LDS) lands in one
    bucket and is sorted by streaming passes over global memory."""
    b = 3 * (1 << 15) + 7
    rng = np.random.default_rng(16)
    note("oversized bucket b=%d" % b)
    t = Trio(b)
    t.g.set_sort_path(LSM.SORT_TOP_DIGIT)
    for r in range(3):
        k = rng.integers(0, 1 << 16, b).astype(np.uint32)
        if r == 2:
            t.delete(k[: b // 2])
        else:
            t.insert(k, rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
        t.check_levels()
    q = np.arange(0, 1 << 16, 7, dtype=np.uint32)
    t.check_queries(q, q[:500], q[:500] + 300)


def test_sort_path_follows_key_skew():
    """Automatic path choice: skewed batches (one key in 70 % of the slots)
    move the sort to digit passes from the next batch on, uniform batches
    move it back; every batch's level layout stays byte-exact either way."""
    b = (1 << 15) + 5
    rng = np.random.default_rng(61)
    note("sort path follows skew b=%d" % b)
    t = Trio(b)
    paths = []
    for r in range(7):
        if r < 3:
            k = rng.integers(0, 1 << 31, b, dtype=np.uint64).astype(np.uint32)
            k[rng.random(b) < 0.7] = 123456789
        else:
            k = rng.integers(0, 1 << 31, b, dtype=np.uint64).astype(np.uint32)
        before = t.g.stats()
        t.insert(k, rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
        t.check_levels()  # synchronises, so the next choice sees this sort
        after = t.g.stats()
        paths.append("top" if after.sorts_top_digit > before.sorts_top_digit else "passes")
    assert paths == ["top", "passes", "passes", "passes", "top", "top", "top"], paths


@pytest.mark.parametrize("mode", [LSM.SORT_TOP_DIGIT, LSM.SORT_DIGIT_PASSES])
def test_forced_sort_paths(mode):
    """Either path, forced, on batches of 1 to 256 tiles (the top-digit
    sort's limit) with partial batches: top-digit buckets sorted by ranking
    (up to 256 elements), by LDS radix passes (about 500 at 255 tiles) and,
    with keys below 2^12 (one bucket), by the streaming fallback.  A forced
    top-digit sort above 256 tiles runs the digit passes (600 tiles)."""
    for b, domain, R, seed in [(1, 8, 20, 71), (2047, 3000, 9, 72), (4096 * 3 + 1, 1 << 31, 6, 73),
                               (255 * 2048 - 9, 1 << 31, 3, 74), ((1 << 19) - 3, 1 << 31, 2, 75),
                               (200 * 2048 + 5, 1 << 12, 2, 76), (600 * 2048 - 9, 1 << 31, 2, 77)]:
        ops, q, lo, hi = W.random_small(seed, b, R, domain, p_delete=0.3, nq=300)
        note("forced sort path %d b=%d" % (mode, b))
        t = Trio(b)
        t.g.set_sort_path(mode)
        for kind, k, v in ops:
            if kind == "insert":
                t.insert(k, v)
            else:
                t.delete(k)
        t.check_levels()
        t.check_queries(q, lo, hi)


@pytest.mark.parametrize("key_bits,b", [(1, 3000), (4, 3000), (9, 2049), (9, 40000)])
def test_few_key_bits(key_bits, b):
    """Keys below 2^key_bits with key_bits under the top digit's 10 bits:
    the top digit then holds every key bit, so a bucket is sorted with no
    digit pass (equal key variables keep their batch order), mixed batches
    put the status bit into the top digit, and most of the 1024 buckets stay
    empty while the others hold many copies of one key.  Partial, deleting
    and mixed batches through the pipelined insertion (pairs, fusion) and
    the automatic path choice; levels byte for byte against the cascade
    oracle, answers against the map oracle."""
    note("few key bits: key_bits=%d b=%d" % (key_bits, b))
    R = 23 if b > 10000 else 37
    ops, _, _, _ = W.random_small(3300 + key_bits, b, R, 1 << key_bits, p_delete=0.3, nq=10)
    t = Trio(b, key_bits=key_bits, checked=True)
    rng = np.random.default_rng(key_bits)
    for i, (kind, k, v) in enumerate(ops):
        if i % 5 == 4:
            vv = v if v is not None else k
            t.mixed(k, vv, (rng.random(k.size) < 0.5).astype(np.uint8))
        elif kind == "insert":
            t.insert(k, v)
        else:
            t.delete(k)
    t.check_levels()
    top = (1 << key_bits) - 1
    q = np.arange(top + 3, dtype=np.uint32)
    lo = np.arange(top + 1, dtype=np.uint32)
    hi = np.minimum(lo + 1 + top // 3, top + 1).astype(np.uint32)
    t.check_queries(q, lo, hi)
    t.check_order(q)
    t.g.close()
