"""Brute-force references used to pin the oracle (test infrastructure).

Each function here is a second, deliberately different way of writing down
what the paper fixes, small enough to check by eye:

* :class:`LogBrute` keeps the raw operation log and answers every query by
  scanning it backwards (sec. III-A batch semantics), never holding a map.
* :func:`closed_form_levels` gives the content of every level without running
  the cascade: level i holds the batches numbered [base, base + 2^i) with
  base = (r >> (i+1)) << (i+1) (the binary-counter picture of sec. III-B),
  ordered by original key, then newest batch first, then tombstone first,
  then later batch position first (building invariants of sec. III-D).
* :func:`cleanup_layout` gives the levels right after a cleanup (sec. III-E,
  IV-D) straight from the live set: its pairs in key order as regular
  elements, padded with placebo tombstones of key 2^31 - 1 to a multiple of b,
  then cut into the levels of the new batch count, smallest level first.
* :func:`lookup_over_levels` / :func:`count_over_levels` /
  :func:`range_over_levels` read a layout the way sec. III-D and III-E (with
  the five count stages of sec. IV-C) describe, so a layout that breaks the
  invariants returns a stale answer.
"""
from __future__ import annotations

import bisect


class LogBrute:
    """Operation log; queries scan it from the newest batch backwards."""

    def __init__(self):
        self.batches = []  # each: list of (key, val, is_delete) in batch order

    def insert(self, keys, vals):
        self.batches.append([(int(k), int(v), False) for k, v in zip(keys, vals)])

    def delete(self, keys):
        self.batches.append([(int(k), 0, True) for k in keys])

    def mixed(self, keys, vals, is_delete):
        self.batches.append([(int(k), int(v), bool(d)) for k, v, d in zip(keys, vals, is_delete)])

    def lookup(self, k):
        k = int(k)
        for batch in reversed(self.batches):
            ops = [(v, d) for (kk, v, d) in batch if kk == k]
            if not ops:
                continue
            if any(d for _, d in ops):          # rule 5: inserted and deleted -> deleted
                return 0, 0
            return ops[-1][0], 1                # last insert in batch order wins
        return 0, 0

    def count(self, k1, k2, domain):
        if k1 > k2:
            return 0
        return sum(self.lookup(k)[1] for k in range(int(k1), min(int(k2), domain - 1) + 1))

    def successor(self, k, domain):
        """Smallest live key > k (scanning the domain upwards), or None."""
        for x in range(int(k) + 1, domain):
            v, f = self.lookup(x)
            if f:
                return x, v
        return None

    def predecessor(self, k, domain):
        """Largest live key < k (scanning the domain downwards), or None."""
        for x in range(min(int(k), domain) - 1, -1, -1):
            v, f = self.lookup(x)
            if f:
                return x, v
        return None

    def live(self, domain):
        return [(k, self.lookup(k)[0]) for k in range(domain) if self.lookup(k)[1]]

    def range(self, k1, k2, domain):
        out = []
        if k1 > k2:
            return out
        for k in range(int(k1), min(int(k2), domain - 1) + 1):
            v, f = self.lookup(k)
            if f:
                out.append((k, v))
        return out


def closed_form_levels(batches, b, status_in_sort=True):
    """batches: list of (keys, vals_or_None, status_list) as inserted, each of
    1..b elements.  Returns {level: [(kv, val), ...]} for occupied levels.
    status_in_sort=False is the coalesced-batch order: inside a batch the
    later position comes first whatever the status."""
    padded = []
    for keys, vals, status in batches:
        n = len(keys)
        row = []
        for p in range(b):
            src = p if p < n else n - 1          # pad with copies of the last element
            s = int(status[src])
            v = int(vals[src]) if (s and vals is not None) else 0
            row.append((int(keys[src]), s, v, p))
        padded.append(row)
    r = len(padded)
    levels = {}
    i = 0
    while (r >> i) != 0:
        if (r >> i) & 1:
            base = (r >> (i + 1)) << (i + 1)
            elems = []
            for t in range(base, base + (1 << i)):
                for (k, s, v, p) in padded[t]:
                    elems.append((k, -t, s if status_in_sort else 0, -p, s, v))
            elems.sort()
            levels[i] = [((k << 1) | s, v) for (k, _t, _s, _p, s, v) in elems]
        i += 1
    return levels


PLACEBO_KV = 0xFFFFFFFE                          # key 2^31 - 1, tombstone


def cleanup_layout(live, b):
    """live: [(key, val)] ascending by key.  Returns (r, {level: (kv, vals)})."""
    r = -(-len(live) // b)
    flat = [((k << 1) | 1, v) for k, v in live]
    flat += [(PLACEBO_KV, 0)] * (r * b - len(live))
    levels, off, i = {}, 0, 0
    while (r >> i) != 0:
        if (r >> i) & 1:
            part = flat[off:off + (b << i)]
            levels[i] = ([kv for kv, _ in part], [v for _, v in part])
            off += b << i
        i += 1
    assert off == len(flat)
    return r, levels


def lookup_over_levels(levels, k):
    """levels: {i: (kv_list, val_list)}; newest (smallest) level first."""
    for i in sorted(levels):
        kv, vals = levels[i]
        keys = [x >> 1 for x in kv]
        p = bisect.bisect_left(keys, k)
        if p < len(keys) and keys[p] == k:
            if kv[p] & 1:
                return int(vals[p]), 1
            return 0, 0                         # tombstone: stop, not found
    return 0, 0


def _candidates(levels, k1, k2):
    cand = []
    for i in sorted(levels):                    # gather in level order
        kv, vals = levels[i]
        keys = [x >> 1 for x in kv]
        lo = bisect.bisect_left(keys, k1)
        hi = bisect.bisect_right(keys, k2)
        cand.extend((int(kv[p]), int(vals[p])) for p in range(lo, hi))
    cand.sort(key=lambda e: e[0] >> 1)          # stable, status bit ignored
    return cand


def range_over_levels(levels, k1, k2):
    if k1 > k2:
        return []
    out, prev = [], None
    for kv, v in _candidates(levels, k1, k2):
        k = kv >> 1
        if k != prev and (kv & 1):              # first of a run, and regular
            out.append((k, v))
        prev = k
    return out


def count_over_levels(levels, k1, k2):
    return len(range_over_levels(levels, k1, k2))
