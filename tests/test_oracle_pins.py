"""Pins of the CPU oracle against what the paper and plain mathematics fix.

CPU only.  Each test checks the oracle against something other than itself:
brute force on tiny key domains, a closed form of the level layout, the
worked cascade of Fig. 1, the building invariants of sec. III-D, the
merge-cost closed form of sec. V-B, and special cases that reduce to a
sorted array (the single-level case of sec. V-A).
"""
import bisect
import os

import numpy as np
import pytest

import oracle
from _brute import (PLACEBO_KV, LogBrute, cleanup_layout, closed_form_levels,
                    count_over_levels, lookup_over_levels, range_over_levels)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_ops(rng, b, nbatch, domain, p_delete=0.3, p_mixed=0.0, partial=True):
    ops = []
    for _ in range(nbatch):
        n = int(rng.integers(1, b + 1)) if partial else b
        keys = rng.integers(0, domain, n).astype(np.uint32)
        vals = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        u = rng.random()
        if u < p_mixed:
            dele = (rng.random(n) < 0.4).astype(np.uint8)
            ops.append(("mixed", keys, vals, dele))
        elif u < p_mixed + p_delete:
            ops.append(("delete", keys, None, None))
        else:
            ops.append(("insert", keys, vals, None))
    return ops


def _apply(ops, b):
    m, brute, casc = oracle.MapOracle(), LogBrute(), oracle.CascadeOracle(b)
    hist = []
    for kind, keys, vals, dele in ops:
        if kind == "insert":
            m.insert(keys, vals); brute.insert(keys, vals); casc.insert(keys, vals)
            hist.append((keys, vals, [1] * len(keys)))
        elif kind == "delete":
            m.delete(keys); brute.delete(keys); casc.delete(keys)
            hist.append((keys, None, [0] * len(keys)))
        else:
            m.mixed(keys, vals, dele); brute.mixed(keys, vals, dele)
            st = (1 - dele).astype(np.uint8)
            casc.insert(keys, vals, st)
            hist.append((keys, vals, list(st)))
    return m, brute, casc, hist


def _layout(casc):
    return {i: tuple(a.tolist() for a in casc.level(i)) for i in casc.occupied()}


# ---------------------------------------------------------------- MapOracle
@pytest.mark.parametrize("b", [1, 2, 3, 4, 8])
def test_map_oracle_vs_log_brute(b):
    domain = 16
    for seed in range(60):
        rng = np.random.default_rng(1000 * b + seed)
        ops = _rand_ops(rng, b, int(rng.integers(1, 13)), domain, p_mixed=0.2)
        m, brute, _, _ = _apply(ops, b)
        q = np.arange(domain + 2, dtype=np.uint32)
        vals, found = m.lookup(q)
        for k in range(domain + 2):
            assert (int(vals[k]), int(found[k])) == brute.lookup(k), (b, seed, k)
        lo = rng.integers(0, domain + 2, 40).astype(np.uint32)
        hi = rng.integers(0, domain + 2, 40).astype(np.uint32)
        cnt = m.count(lo, hi)
        off, rk, rv = m.range(lo, hi)
        for j in range(40):
            want = brute.range(lo[j], hi[j], domain + 2)
            assert int(cnt[j]) == len(want) == brute.count(lo[j], hi[j], domain + 2)
            got = list(zip(rk[off[j]:off[j + 1]].tolist(), rv[off[j]:off[j + 1]].tolist()))
            assert got == want, (b, seed, j)
        assert len(m) == sum(brute.lookup(k)[1] for k in range(domain))


def test_map_oracle_batch_rules():
    """The six batch rules of sec. III-A, each on a hand-made case."""
    m = oracle.MapOracle()
    m.insert([5, 5, 7], [1, 2, 3])                 # rule 3 (reading: last wins)
    assert m.lookup([5, 7])[0].tolist() == [2, 3]
    m.insert([5], [9])                             # rule 3 across batches: newest wins
    assert m.lookup([5])[0].tolist() == [9]
    m.delete([7, 7])                               # rule 4: repeated delete == one delete
    assert m.lookup([7])[1].tolist() == [0]
    m.mixed([8, 8], [4, 0], [0, 1])                # rule 5: inserted and deleted -> deleted
    assert m.lookup([8])[1].tolist() == [0]
    m.mixed([9, 9], [0, 6], [1, 0])                # delete listed first, still deleted
    assert m.lookup([9])[1].tolist() == [0]
    assert m.count([0], [100]).tolist() == [1]     # only key 5 is live
    assert m.count([6], [5]).tolist() == [0]       # k1 > k2 -> 0
    assert m.count([5], [5]).tolist() == [1]       # bounds are inclusive


# ------------------------------------------------------------ CascadeOracle
@pytest.mark.parametrize("b", [1, 2, 3, 4, 8])
def test_cascade_oracle_vs_closed_form(b):
    for seed in range(40):
        rng = np.random.default_rng(7000 + 100 * b + seed)
        ops = _rand_ops(rng, b, int(rng.integers(1, 13)), 16, p_mixed=0.2)
        _, _, casc, hist = _apply(ops, b)
        want = closed_form_levels(hist, b)
        got = _layout(casc)
        assert casc.r == len(hist)
        assert sorted(got) == sorted(want)
        for i in want:
            assert list(zip(*got[i])) == want[i], (b, seed, i)


@pytest.mark.parametrize("b", [1, 2, 3, 4, 8])
def test_layout_answers_match_map_oracle(b):
    """Reading the layout as sec. III-D/III-E prescribe gives the dictionary
    answers: any tie or placement mistake in the cascade returns a stale
    value or a deleted key here."""
    domain = 16
    for seed in range(40):
        rng = np.random.default_rng(9000 + 100 * b + seed)
        ops = _rand_ops(rng, b, int(rng.integers(1, 13)), domain, p_mixed=0.2)
        m, _, casc, _ = _apply(ops, b)
        levels = _layout(casc)
        vals, found = m.lookup(np.arange(domain, dtype=np.uint32))
        for k in range(domain):
            assert lookup_over_levels(levels, k) == (int(vals[k]), int(found[k]))
        for k1 in range(domain):
            for k2 in range(k1 - 1, domain):
                off, rk, rv = m.range([k1], [max(k2, 0)])
                if k2 < k1:
                    assert count_over_levels(levels, k1, k2) == 0
                    continue
                got = range_over_levels(levels, k1, k2)
                assert got == list(zip(rk.tolist(), rv.tolist()))
                assert count_over_levels(levels, k1, k2) == int(m.count([k1], [k2])[0])


def test_fig1_cascade_shape():
    spec = {}
    with open(os.path.join(GOLDEN, "fig1_cascade.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, *v = line.split()
                spec[k] = [int(x) for x in v]
    b = 4
    casc = oracle.CascadeOracle(b)
    rng = np.random.default_rng(1)
    for _ in range(spec["r_before"][0]):
        casc.insert(rng.integers(0, 2**31, b).astype(np.uint32),
                    rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
    assert casc.occupied() == spec["occupied_before"]
    untouched = {i: casc.level(i) for i in spec["untouched_levels"]}
    casc.insert(rng.integers(0, 2**31, b).astype(np.uint32),
                rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
    assert casc.r == spec["r_after"][0]
    assert casc.occupied() == spec["occupied_after"]
    assert casc.merged_last == spec["merged_elements_in_units_of_b"][0] * b
    for i, (kv, v) in untouched.items():
        kv2, v2 = casc.level(i)
        assert np.array_equal(kv, kv2) and np.array_equal(v, v2)
    for i in casc.occupied():
        assert casc.level(i)[0].size == b << i


@pytest.mark.parametrize("b", [1, 3, 16])
def test_building_invariants(b):
    """Sec. III-D invariants 1 and 2 plus the binary-counter occupancy of
    sec. III-B.  Values encode (batch, position) so recency is visible."""
    rng = np.random.default_rng(b)
    casc = oracle.CascadeOracle(b)
    for t in range(37):
        keys = rng.integers(0, 8, b).astype(np.uint32)
        vals = (t << 16) + np.arange(b, dtype=np.uint32)
        casc.insert(keys, vals)
        assert casc.r == t + 1
        occ = casc.occupied()
        assert occ == [i for i in range(8) if ((t + 1) >> i) & 1]
        assert sum(casc.level(i)[0].size for i in occ) == (t + 1) * b
        assert all(casc.level(i)[0].size == 0 for i in range(8) if i not in occ)
        for i in occ:
            kv, v = casc.level(i)
            k = kv >> 1
            assert np.all(k[1:] >= k[:-1])                           # invariant 1
            same = k[1:] == k[:-1]
            assert np.all((v[1:] >> 16)[same] <= (v[:-1] >> 16)[same])  # invariant 2
            within = same & ((v[1:] >> 16) == (v[:-1] >> 16))
            assert np.all((v[1:] & 0xFFFF)[within] < (v[:-1] & 0xFFFF)[within])


def test_mixed_batch_exact_layout():
    """Sec. III-D invariant 3 inside one mixed batch: the tombstone precedes
    the regular elements of its key."""
    casc = oracle.CascadeOracle(4)
    casc.insert([3, 3, 3, 1], [10, 0, 11, 5], [1, 0, 1, 1])
    kv, v = casc.level(0)
    # padded to b=4 already (n == b); order: key 1, then key 3 tombstone, then
    # key 3 regular elements latest position first.
    assert kv.tolist() == [3, 6, 7, 7]
    assert v.tolist() == [5, 0, 11, 10]


@pytest.mark.parametrize("b", [1, 2, 5, 8])
def test_merge_cost_closed_form(b):
    """Merged elements per insertion = (2^(ffz(r)+1) - 2) b: the merge term of
    T_ins(r) in sec. V-B counted in elements written."""
    casc = oracle.CascadeOracle(b)
    rng = np.random.default_rng(3)
    for r in range(70):
        casc.insert(rng.integers(0, 100, b).astype(np.uint32), np.zeros(b, np.uint32))
        ffz = (~r & (r + 1)).bit_length() - 1
        assert casc.merged_last == ((1 << (ffz + 1)) - 2) * b


def test_single_level_is_sorted_array():
    """b >= all elements: one level, i.e. a sorted array; lookup reduces to a
    textbook lower bound (the single-level case of sec. V-A)."""
    rng = np.random.default_rng(11)
    keys = rng.choice(2**31, 5000, replace=False).astype(np.uint32)
    vals = rng.integers(0, 2**32, 5000, dtype=np.uint64).astype(np.uint32)
    casc = oracle.CascadeOracle(5000)
    casc.insert(keys, vals)
    kv, v = casc.level(0)
    order = np.argsort(keys)
    assert np.array_equal(kv >> 1, keys[order]) and np.all(kv & 1)
    assert np.array_equal(v, vals[order])
    m = oracle.MapOracle()
    m.insert(keys, vals)
    q = np.concatenate([keys[:500], rng.integers(0, 2**31, 500).astype(np.uint32)])
    got_v, got_f = m.lookup(q)
    sk = (kv >> 1).tolist()
    for j, k in enumerate(q.tolist()):
        p = bisect.bisect_left(sk, k)
        hit = p < len(sk) and sk[p] == k
        assert got_f[j] == hit and (not hit or got_v[j] == v[p])


def test_count_without_duplicates_is_sum_of_bound_differences():
    """No deletes and distinct keys: count = sum over levels of
    upper_bound(k2) - lower_bound(k1) (sec. III-E)."""
    rng = np.random.default_rng(5)
    b = 64
    allk = rng.choice(2**20, 64 * 13, replace=False).astype(np.uint32)
    casc, m = oracle.CascadeOracle(b), oracle.MapOracle()
    for t in range(13):
        k = allk[t * b:(t + 1) * b]
        casc.insert(k, k)
        m.insert(k, k)
    lo = rng.integers(0, 2**20, 200).astype(np.uint32)
    hi = (lo + rng.integers(0, 2**16, 200)).astype(np.uint32)
    cnt = m.count(lo, hi)
    for j in range(200):
        s = 0
        for i in casc.occupied():
            keys = casc.level(i)[0] >> 1
            s += int(np.searchsorted(keys, hi[j], "right") - np.searchsorted(keys, lo[j], "left"))
        assert s == int(cnt[j])


def test_partial_batch_padding_is_invisible():
    """A partial batch padded with copies of its last element answers like
    the unpadded batch (sec. IV-A), even when the last key also appears
    earlier in the batch."""
    casc, m = oracle.CascadeOracle(8), oracle.MapOracle()
    casc.insert([4, 2, 4], [1, 2, 3])
    m.insert([4, 2, 4], [1, 2, 3])
    levels = _layout(casc)
    assert lookup_over_levels(levels, 4) == (3, 1)
    assert lookup_over_levels(levels, 2) == (2, 1)
    assert tuple(a.tolist()[0] for a in m.lookup([4])) == (3, 1)
    assert casc.level(0)[0].size == 8


def _pack(user_batches, b):
    """Coalesce single-type user batches, in arrival order, into batches of
    b: returns list of (keys, vals, status) with the last one partial."""
    k = np.concatenate([u[0] for u in user_batches]).astype(np.uint32)
    v = np.concatenate([u[1] for u in user_batches]).astype(np.uint32)
    s = np.concatenate([np.full(u[0].size, 0 if u[2] else 1, np.uint8) for u in user_batches])
    return [(k[o:o + b], v[o:o + b], s[o:o + b]) for o in range(0, k.size, b)]


@pytest.mark.parametrize("b", [1, 3, 8])
def test_coalesced_batches_match_sequential_user_batches(b):
    """Packing user batches into LSM batches keeps their meaning: the
    ordered-batch layout read as sec. III-D prescribes answers like the user
    batches applied one after another, and equals its closed form."""
    domain = 12
    for seed in range(60):
        rng = np.random.default_rng(40000 + 100 * b + seed)
        m = oracle.MapOracle()
        users = []
        for _ in range(int(rng.integers(1, 15))):
            n = int(rng.integers(1, 2 * b + 2))
            k = rng.integers(0, domain, n).astype(np.uint32)
            v = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
            dele = bool(rng.random() < 0.35)
            users.append((k, v, dele))
            if dele:
                m.delete(k)
            else:
                m.insert(k, v)
        casc = oracle.CascadeOracle(b)
        hist = []
        for (k, v, s) in _pack(users, b):
            casc.insert_ordered(k, v, s)
            hist.append((k, v, list(s)))
        levels = _layout(casc)
        want = closed_form_levels(hist, b, status_in_sort=False)
        assert sorted(levels) == sorted(want)
        for i in want:
            assert list(zip(*levels[i])) == want[i]
        vals, found = m.lookup(np.arange(domain, dtype=np.uint32))
        for key in range(domain):
            assert lookup_over_levels(levels, key) == (int(vals[key]), int(found[key])), (b, seed, key)
        for k1 in range(domain):
            k2 = min(domain - 1, k1 + 3)
            assert count_over_levels(levels, k1, k2) == int(m.count([k1], [k2])[0])


def test_coalesced_insert_after_delete_in_one_batch():
    """The case that separates the two batch orders: a delete then a later
    insert of the same key inside one packed batch leaves the key present."""
    casc = oracle.CascadeOracle(4)
    casc.insert_ordered([5, 5, 2, 7], [0, 99, 1, 2], [0, 1, 1, 1])
    assert lookup_over_levels(_layout(casc), 5) == (99, 1)
    casc2 = oracle.CascadeOracle(4)
    casc2.insert([5, 5, 2, 7], [0, 99, 1, 2], [0, 1, 1, 1])
    assert lookup_over_levels(_layout(casc2), 5) == (0, 0)


# ------------------------------------------------------------ order queries
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_successor_predecessor_vs_log_brute(seed):
    rng = np.random.default_rng(500 + seed)
    domain = 24
    ops = _rand_ops(rng, 4, 10, domain, p_delete=0.35, p_mixed=0.1)
    m, brute, _c, _h = _apply(ops, 4)
    q = np.arange(0, domain + 3, dtype=np.uint32)
    sk, sv, sf = m.successor(q)
    pk, pv, pf = m.predecessor(q)
    for i, k in enumerate(q.tolist()):
        s = brute.successor(k, domain)
        assert (int(sf[i]), int(sk[i]), int(sv[i])) == ((1, s[0], s[1]) if s else (0, 0, 0)), k
        p = brute.predecessor(k, domain)
        assert (int(pf[i]), int(pk[i]), int(pv[i])) == ((1, p[0], p[1]) if p else (0, 0, 0)), k


def test_order_queries_at_the_ends_of_the_key_space():
    m = oracle.MapOracle()
    top = 2**31 - 1
    m.insert([0, 5, top], [10, 50, 70])
    k, v, f = m.successor([top, top - 1, 0, 2**32 - 1])
    assert f.tolist() == [0, 1, 1, 0] and k.tolist() == [0, top, 5, 0] and v.tolist() == [0, 70, 50, 0]
    k, v, f = m.predecessor([0, 1, 6, 2**32 - 1])
    assert f.tolist() == [0, 1, 1, 1] and k.tolist() == [0, 0, 5, top] and v.tolist() == [0, 10, 50, 70]


# ------------------------------------------------------------ cleanup
def _cleanup_case(seed, b, nbatch, domain):
    rng = np.random.default_rng(seed)
    ops = _rand_ops(rng, b, nbatch, domain, p_delete=0.3, p_mixed=0.1)
    return _apply(ops, b)


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5])
def test_cleanup_layout_is_the_live_set_sliced(b):
    for seed in range(8):
        m, brute, casc, _h = _cleanup_case(700 + 10 * b + seed, b, 9 + seed, 20)
        live = brute.live(20)
        v = casc.cleanup()
        assert v == len(live) == len(m)
        r, expect = cleanup_layout(live, b)
        assert casc.r == r
        assert _layout(casc) == {i: (kv, vals) for i, (kv, vals) in expect.items()}
        for i in range(64):
            if i not in expect:
                assert casc.level(i)[0].size == 0


@pytest.mark.parametrize("b", [2, 3, 4])
def test_cleanup_keeps_every_answer_and_later_batches_still_work(b):
    domain = 20
    for seed in range(6):
        rng = np.random.default_rng(900 + 7 * b + seed)
        ops = _rand_ops(rng, b, 11, domain, p_delete=0.3, p_mixed=0.1)
        m, brute, casc, _h = _apply(ops, b)
        casc.cleanup()
        more = _rand_ops(rng, b, 7, domain, p_delete=0.3, p_mixed=0.1)
        for step in range(len(more) + 1):
            lay = {i: casc.level(i) for i in casc.occupied()}
            lay = {i: (kv.tolist(), v.tolist()) for i, (kv, v) in lay.items()}
            for k in range(domain):
                assert lookup_over_levels(lay, k) == brute.lookup(k), (seed, step, k)
            for k1 in range(0, domain, 3):
                for k2 in range(k1, domain + 2, 4):
                    assert range_over_levels(lay, k1, k2) == brute.range(k1, k2, domain)
            for i, (kv, _v) in lay.items():
                keys = [x >> 1 for x in kv]
                assert keys == sorted(keys) and len(kv) == b << i
            if step == len(more):
                break
            kind, keys, vals, dele = more[step]
            if kind == "insert":
                brute.insert(keys, vals); casc.insert(keys, vals)
            elif kind == "delete":
                brute.delete(keys); casc.delete(keys)
            else:
                brute.mixed(keys, vals, dele); casc.insert(keys, vals, (1 - dele).astype(np.uint8))


def test_cleanup_structure_properties():
    """No stale element survives, placebos are fewer than b and sit at the end
    of the largest level, and smaller keys lie in smaller levels."""
    b = 8
    m, brute, casc, _h = _cleanup_case(31, b, 40, 200)
    casc.cleanup()
    occ = casc.occupied()
    assert occ and casc.r == -(-len(m) // b)
    prev_max = -1
    placebos = 0
    for i in occ:
        kv, v = casc.level(i)
        real = kv[kv != PLACEBO_KV]
        if i != occ[-1]:
            assert real.size == kv.size
        else:
            tail = kv[real.size:]
            assert np.all(tail == PLACEBO_KV) and np.all(v[real.size:] == 0)
            placebos = tail.size
        assert np.all(real & 1 == 1)
        keys = (real >> 1).astype(np.int64)
        assert np.all(np.diff(keys) > 0)
        assert keys.size == 0 or keys[0] > prev_max
        if keys.size:
            prev_max = keys[-1]
    assert placebos < b
    assert placebos == casc.r * b - len(m)


def test_cleanup_special_cases():
    b = 4
    c = oracle.CascadeOracle(b)
    assert c.cleanup() == 0 and c.r == 0 and c.occupied() == []
    c.insert([1, 2, 3], [7, 8, 9])
    c.delete([3, 2, 1])
    assert c.cleanup() == 0 and c.r == 0 and c.occupied() == []
    # A live key 2^31 - 1 is not hidden by the placebos of its own key.
    top = 2**31 - 1
    c.insert([top, 4], [11, 12])
    assert c.cleanup() == 2 and c.r == 1
    kv, v = c.level(0)
    assert kv.tolist() == [(4 << 1) | 1, (top << 1) | 1, PLACEBO_KV, PLACEBO_KV]
    assert v.tolist() == [12, 11, 0, 0]
    lay = {0: (kv.tolist(), v.tolist())}
    assert lookup_over_levels(lay, top) == (11, 1)
    assert count_over_levels(lay, 0, top) == 2
    # After a newer delete of that key, it is gone.
    c.delete([top])
    lay = {i: tuple(a.tolist() for a in c.level(i)) for i in c.occupied()}
    assert lookup_over_levels(lay, top) == (0, 0)
    assert count_over_levels(lay, 0, top) == 1
