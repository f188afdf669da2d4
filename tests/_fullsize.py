"""Host helpers of the full-size parity tests (no GPU work here).

A dictionary's answer for a key depends only on the operations on that key,
so the map oracle fed, in order, only the operations whose keys can affect a
sample of queries answers exactly those queries without holding the whole
workload.  `key_filter` builds the membership test for a sample, and
`FilteredMap` applies operations through it."""
from __future__ import annotations

import numpy as np

import oracle


def key_filter(points=(), lo=(), hi=()):
    """keep(keys) -> bool mask: keys equal to one of `points` or inside one of
    the inclusive intervals [lo[i], hi[i]]."""
    lo = np.concatenate([np.asarray(points, np.int64), np.asarray(lo, np.int64)])
    hi = np.concatenate([np.asarray(points, np.int64), np.asarray(hi, np.int64)])
    order = np.argsort(lo, kind="stable")
    slo, shi = lo[order], hi[order]
    run_hi = np.maximum.accumulate(shi) if shi.size else shi

    def keep(k):
        k = np.asarray(k).astype(np.int64)
        if slo.size == 0:
            return np.zeros(k.shape, bool)
        j = np.searchsorted(slo, k, side="right") - 1
        return (j >= 0) & (k <= run_hi[np.maximum(j, 0)])
    return keep


class FilteredMap:
    """Map oracle fed only the operations whose key passes keep()."""

    def __init__(self, keep):
        self.keep = keep
        self.m = oracle.MapOracle()

    def insert(self, keys, vals):
        sel = self.keep(keys)
        if sel.any():
            self.m.insert(np.asarray(keys)[sel], np.asarray(vals)[sel])

    def delete(self, keys):
        sel = self.keep(keys)
        if sel.any():
            self.m.delete(np.asarray(keys)[sel])

    def mixed_in_order(self, keys, vals, is_del):
        """Operations of both types in arrival order (runs of one type are
        applied as one batch, element by element)."""
        keys, vals, is_del = np.asarray(keys), np.asarray(vals), np.asarray(is_del).astype(bool)
        sel = self.keep(keys)
        keys, vals, is_del = keys[sel], vals[sel], is_del[sel]
        if keys.size == 0:
            return
        cut = np.flatnonzero(np.diff(is_del.astype(np.int8))) + 1
        for a, e in zip(np.r_[0, cut], np.r_[cut, keys.size]):
            if is_del[a]:
                self.m.delete(keys[a:e])
            else:
                self.m.insert(keys[a:e], vals[a:e])


def ranges_of(roff, rk, rv, idx):
    """Concatenated (keys, vals) and sizes of the range queries idx."""
    roff = np.asarray(roff).astype(np.int64)
    ks = np.concatenate([rk[roff[j]:roff[j + 1]] for j in idx]) if len(idx) else rk[:0]
    vs = np.concatenate([rv[roff[j]:roff[j + 1]] for j in idx]) if len(idx) else rv[:0]
    return ks, vs, np.diff(roff)[idx]


def check_range_properties(lo, hi, roff, rk, counts=None):
    """Properties of any range answer: offsets non-decreasing, keys inside
    their query's bounds and strictly ascending within a query, and (when
    given) sizes equal to the counts of the same queries."""
    roff = np.asarray(roff).astype(np.int64)
    sizes = np.diff(roff)
    assert np.all(sizes >= 0) and roff[0] == 0 and roff[-1] == rk.size
    if counts is not None:
        assert np.array_equal(sizes, np.asarray(counts).astype(np.int64)), "count != range size"
    qid = np.repeat(np.arange(lo.size), sizes)
    assert np.all(rk >= lo[qid]) and np.all(rk <= hi[qid]), "range key outside its bounds"
    same_q = qid[1:] == qid[:-1]
    assert np.all(rk[1:][same_q] > rk[:-1][same_q]), "range keys not strictly ascending"


def ops_touching(keys, points=(), lo=(), hi=()):
    """Indices, in operation order, of the operations (keys[i] is the key of
    operation i) whose key equals one of `points` or lies inside one of the
    inclusive intervals [lo[j], hi[j]].  The operations are sorted once by
    (key, index) and each interval's run is cut out of that order, which is
    much faster than testing every key against the sample."""
    keys = np.asarray(keys).reshape(-1)
    z = np.sort((keys.astype(np.uint64) << np.uint64(32)) | np.arange(keys.size, dtype=np.uint64))
    lo = np.concatenate([np.asarray(points, np.uint64), np.asarray(lo, np.uint64)])
    hi = np.concatenate([np.asarray(points, np.uint64), np.asarray(hi, np.uint64)])
    a = np.searchsorted(z, lo << np.uint64(32), side="left")
    e = np.searchsorted(z, (hi + np.uint64(1)) << np.uint64(32), side="left")
    mark = np.zeros(z.size + 1, np.int32)
    np.add.at(mark, a, 1)
    np.add.at(mark, e, -1)
    sel = np.cumsum(mark[:-1]) > 0
    return np.sort((z[sel] & np.uint64(0xFFFFFFFF)).astype(np.int64))
