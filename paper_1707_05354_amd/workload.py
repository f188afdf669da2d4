"""Seeded synthetic inputs for the LSM dictionary (numpy only).

This module produces operation streams and query sets; it holds none of the
dictionary's arithmetic (no sorting, merging or query answering) and is the
only code shared by the oracle side and the GPU side of the tests.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw i of stream (c, s) is mix64(seed + (i + 1) * GAMMA) with
seed = (c << 32) | s, so any slice of a stream can be generated on its own.
Streams: 1 keys, 2 values, 3 delete-key picks, 4 lookup picks, 5 count/range
starts, 6 lookup miss keys, 7 Zipf draws, 8 batch sizes, 9 request mix.

The paper's workloads are uniformly random 31-bit keys (sec. V-B, V-C); the
recipes below follow that, and the Zipf recipe stands in for the skewed
reinsertion workload that exercises stale and tombstoned elements.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
KEY_DOMAIN = 1 << 31


def splitmix64(config: int, stream: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of stream (config, stream) as uint64."""
    seed = np.uint64(((config & 0xFFFFFFFF) << 32) | (stream & 0xFFFFFFFF))
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = seed + i * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_keys(config: int, stream: int, start: int, n: int, bits: int = 31) -> np.ndarray:
    return (splitmix64(config, stream, start, n) >> np.uint64(64 - bits)).astype(np.uint32)


def values(config: int, stream: int, start: int, n: int) -> np.ndarray:
    return (splitmix64(config, stream, start, n) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def bounded(config: int, stream: int, start: int, n: int, bound: int) -> np.ndarray:
    """Integers in [0, bound) (multiply-shift on the top 32 bits)."""
    x = splitmix64(config, stream, start, n) >> np.uint64(32)
    return ((x * np.uint64(bound)) >> np.uint64(32)).astype(np.int64)


@dataclass
class PlainWorkload:
    """A build of R update batches of b slots followed by three query sets.

    keys/vals: uint32 [R, b]; is_delete: bool [R] (a delete batch's values are
    unused).  Queries: lookups [nq], count_lo/hi and range_lo/hi [nc].
    """
    name: str
    b: int
    keys: np.ndarray
    vals: np.ndarray
    is_delete: np.ndarray
    lookups: np.ndarray
    count_lo: np.ndarray
    count_hi: np.ndarray
    range_lo: np.ndarray
    range_hi: np.ndarray
    width: int
    key_bits: int = 31
    meta: dict = field(default_factory=dict)

    @property
    def R(self) -> int:
        return int(self.keys.shape[0])


def _delete_batch_keys(config, keys, is_delete, b):
    """Fill each delete batch with keys drawn, with replacement, from all keys
    inserted by earlier insert batches."""
    ins_rows: List[int] = []
    draw = 0
    for i in range(keys.shape[0]):
        if not is_delete[i]:
            ins_rows.append(i)
            continue
        pool = len(ins_rows) * b
        assert pool > 0, "a delete batch needs earlier inserts"
        idx = bounded(config, 3, draw, b, pool)
        draw += b
        rows = np.asarray(ins_rows, dtype=np.int64)[idx // b]
        keys[i] = keys[rows, idx % b]


def _key_classes(flat, bidx, dele):
    """Classes of a stream's keys fixed by the stream itself, by set
    membership alone.  flat: the keys of every operation in order, bidx:
    each operation's batch number (non-decreasing), dele: whether it
    deletes.  Returns `sure_live`, inserted keys that no deletion names
    (present at the end whatever the order of operations), `sure_dead`,
    deleted keys all of whose insertions come before their first deletion
    (absent at the end), and `inserted`, every inserted key (sorted,
    distinct)."""
    flat = flat.astype(np.uint64)
    bidx = bidx.astype(np.uint64)
    ins = ~dele
    # (key, batch) packed in 64 bits and sorted: per key, batches ascending.
    iz = np.sort((flat[ins] << np.uint64(32)) | bidx[ins])
    ik = (iz >> np.uint64(32)).astype(np.uint32)
    last = np.append(ik[1:] != ik[:-1], True)          # last insertion of each key
    inserted, ins_last = ik[last], (iz[last] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    if not dele.any():
        return ik, np.zeros(0, np.uint32), inserted
    dz = np.sort((flat[dele] << np.uint64(32)) | bidx[dele])
    dk = (dz >> np.uint64(32)).astype(np.uint32)
    first = np.insert(dk[1:] != dk[:-1], 0, True)       # first deletion of each key
    dkeys, del_first = dk[first], (dz[first] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    j = np.minimum(np.searchsorted(inserted, dkeys), inserted.size - 1)
    had = inserted[j] == dkeys
    sure_dead = dkeys[~had | (ins_last[j] < del_first)]
    j = np.minimum(np.searchsorted(dkeys, ik), dkeys.size - 1)
    return ik[dkeys[j] != ik], sure_dead, inserted


def query_set(config, flat, bidx, dele, nq, ncount, expected_hits, domain=KEY_DOMAIN):
    """Queries over a stream of operations (see _key_classes for the stream's
    arrays).  Lookups: half hits drawn from the keys sure to be present, half
    misses (half of those deleted keys, half keys never inserted).  Count /
    range widths expect `expected_hits` present keys, from the estimated
    number of present keys (inserted keys minus those sure to be deleted).
    Returns (lookups, count_lo, count_hi, range_lo, range_hi, width)."""
    live, dead, inserted = _key_classes(flat, bidx, dele)
    pick = splitmix64(config, 4, 0, nq)
    hit = (pick & np.uint64(1)).astype(bool)
    idx = ((pick >> np.uint64(32)) * np.uint64(live.size)) >> np.uint64(32)
    # Misses: a uniform draw, rejected while it names an inserted key
    # (redrawn from later positions of the stream).
    miss = np.zeros(nq, np.uint32)
    todo = np.arange(nq)
    start = 0
    while todo.size:
        cand = (splitmix64(config, 6, start, todo.size) % np.uint64(domain)).astype(np.uint32)
        start += todo.size
        o = np.argsort(cand)  # sorted probes search much faster
        j = np.empty(cand.size, np.int64)
        j[o] = np.searchsorted(inserted, cand[o])
        clash = (j < inserted.size) & (inserted[np.minimum(j, inserted.size - 1)] == cand)
        miss[todo[~clash]] = cand[~clash]
        todo = todo[clash]
    if dead.size:
        dpick = splitmix64(config, 6, 1 << 40, nq)
        use_dead = (dpick & np.uint64(1)).astype(bool)
        didx = ((dpick >> np.uint64(32)) * np.uint64(dead.size)) >> np.uint64(32)
        miss = np.where(use_dead, dead[didx.astype(np.int64)], miss)
    lookups = np.where(hit, live[idx.astype(np.int64)], miss).astype(np.uint32)
    present = max(1, inserted.size - dead.size)
    width = max(1, int(round(expected_hits * domain / present)))
    starts = bounded(config, 5, 0, 2 * ncount, domain - width + 1).astype(np.uint32)
    c_lo, r_lo = starts[:ncount], starts[ncount:]
    return lookups, c_lo, (c_lo + np.uint32(width - 1)), r_lo, (r_lo + np.uint32(width - 1)), width


def _queries(config, keys, is_delete, nq, ncount, expected_hits, domain):
    """query_set over R batches of b (keys [R, b], is_delete [R])."""
    R, b = keys.shape
    return query_set(config, keys.reshape(-1), np.repeat(np.arange(R), b),
                     np.repeat(is_delete, b), nq, ncount, expected_hits, domain)


def tiny(config: int = 1) -> PlainWorkload:
    """b = 1024: 16 insert batches, then 4 delete batches of keys drawn from
    the inserted ones; 4096 lookups (half hits), 1024 count and 1024 range
    queries whose width expects about 8 hits."""
    b, R = 1024, 20
    is_delete = np.array([False] * 16 + [True] * 4)
    keys = uniform_keys(config, 1, 0, R * b).reshape(R, b)
    vals = values(config, 2, 0, R * b).reshape(R, b)
    _delete_batch_keys(config, keys, is_delete, b)
    lk, clo, chi, rlo, rhi, w = _queries(config, keys, is_delete, 4096, 1024, 8, KEY_DOMAIN)
    return PlainWorkload("tiny b=1024 R=20 (16 insert + 4 delete batches)", b, keys, vals,
                         is_delete, lk, clo, chi, rlo, rhi, w)


def paper_scale(config: int = 2, b: int = 1 << 16, R: int = 1024, nq: int = 1 << 22,
                ncount: int = 1 << 20, expected_hits: int = 16) -> PlainWorkload:
    """b = 2^16, R = 1024 batches (n = 2^26 slots), uniform 31-bit keys;
    batch i deletes iff i mod 10 == 9 (keys drawn from earlier inserts).
    Then 2^22 lookups (half hits), 2^20 count and 2^20 range queries of a
    width that expects 16 hits."""
    is_delete = (np.arange(R) % 10) == 9
    keys = uniform_keys(config, 1, 0, R * b).reshape(R, b)
    vals = values(config, 2, 0, R * b).reshape(R, b)
    _delete_batch_keys(config, keys, is_delete, b)
    lk, clo, chi, rlo, rhi, w = _queries(config, keys, is_delete, nq, ncount, expected_hits, KEY_DOMAIN)
    return PlainWorkload("paper scale b=2^16 R=%d n=%d" % (R, R * b), b, keys, vals,
                         is_delete, lk, clo, chi, rlo, rhi, w)


def random_small(seed: int, b: int, R: int, domain: int, p_delete: float = 0.3,
                 nq: int = 512, partial: bool = True):
    """Small mixed stream for edge-case tests: list of (kind, keys, vals) with
    batch sizes in [1, b] when partial, key domain [0, domain)."""
    ops = []
    off = 0
    sizes = (bounded(seed, 8, 0, R, b) + 1) if partial else np.full(R, b)
    kinds = bounded(seed, 9, 0, R, 1000)
    n_ins = 0
    for t in range(R):
        n = int(sizes[t])
        k = (splitmix64(seed, 1, off, n) % np.uint64(domain)).astype(np.uint32)
        v = values(seed, 2, off, n)
        off += n
        if kinds[t] < p_delete * 1000 and n_ins > 0:
            ops.append(("delete", k, None))
        else:
            ops.append(("insert", k, v))
            n_ins += 1
    q = (splitmix64(seed, 4, 0, nq) % np.uint64(domain + 2)).astype(np.uint32)
    a = (splitmix64(seed, 5, 0, nq) % np.uint64(domain + 2)).astype(np.uint32)
    c = (splitmix64(seed, 6, 0, nq) % np.uint64(domain + 2)).astype(np.uint32)
    return ops, q, np.minimum(a, c), np.maximum(a, c)


# ---------------------------------------------------------------- Zipf sweep
ZIPF_S = 1.1
ZIPF_BITS = 24


def zipf_ranks(config: int, stream: int, start: int, n: int, s: float = ZIPF_S,
               bits: int = ZIPF_BITS, _cache={}) -> np.ndarray:
    """Ranks 1..2^bits drawn from the bounded Zipf law P(k) ~ k^-s by
    inverting its cumulative distribution (numpy float64 cumulative sum,
    deterministic for a given numpy)."""
    key = (s, bits)
    if key not in _cache:
        w = np.arange(1, (1 << bits) + 1, dtype=np.float64) ** (-s)
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        _cache.clear()
        _cache[key] = cdf
    cdf = _cache[key]
    u = (splitmix64(config, stream, start, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, 1 << bits).astype(np.int64)


def zipf_keys(config: int, stream: int, start: int, n: int, bits: int = ZIPF_BITS) -> np.ndarray:
    """Zipf ranks mapped to keys in [0, 2^bits) by a seeded bijection
    (multiply by an odd constant, then XOR a seeded mask), so hot keys are
    spread over the key space."""
    mask_bits = (1 << bits) - 1
    r = zipf_ranks(config, stream, start, n, bits=bits) - 1
    odd = 0x9E3779B1 & mask_bits | 1
    xmask = int(splitmix64(config, 15, 0, 1)[0]) & mask_bits
    return (((r * odd) & mask_bits) ^ xmask).astype(np.uint32)


_ZIPF_STREAM = {}


def _zipf_stream(config: int, n_total: int, nq: int):
    """Keys, values and lookups shared by every sweep point (cached)."""
    k = (config, n_total, nq)
    if k not in _ZIPF_STREAM:
        _ZIPF_STREAM.clear()
        _ZIPF_STREAM[k] = (zipf_keys(config, 1, 0, n_total), values(config, 2, 0, n_total),
                           zipf_keys(config, 4, 0, nq))
    return _ZIPF_STREAM[k]


def zipf_sweep(b: int, config: int = 3, n_total: int = 1 << 25, nq: int = 1 << 22) -> PlainWorkload:
    """Batch-size sweep point: n_total slots in batches of b, keys Zipf(1.1)
    over [0, 2^24) from one shared stream (every sweep point sees the same key
    sequence, cut into batches of its own b), batch i deletes iff
    i mod 5 == 4 (its keys drawn from the same law), then nq Zipf lookups and
    2^16 count / range queries of width 2^8 over the 2^24 key space."""
    R = n_total // b
    keys, vals, lookups = _zipf_stream(config, n_total, nq)
    keys = keys[:R * b].reshape(R, b)
    vals = vals[:R * b].reshape(R, b)
    is_delete = (np.arange(R) % 5) == 4
    nc = 1 << 16
    width = 1 << 8
    starts = bounded(config, 5, 0, 2 * nc, (1 << ZIPF_BITS) - width + 1).astype(np.uint32)
    c_lo, r_lo = starts[:nc], starts[nc:]
    return PlainWorkload("zipf sweep b=%d R=%d n=%d" % (b, R, R * b), b, keys, vals, is_delete,
                         lookups, c_lo, c_lo + np.uint32(width - 1), r_lo,
                         r_lo + np.uint32(width - 1), width, key_bits=ZIPF_BITS)


# ---------------------------------------------------------------- batching
def cleanup_build(b: int, R: int, stale: float, config: int = 6, nq: int = 1 << 22):
    """R insert batches of b uniform 31-bit keys in which each element, with
    probability `stale`, re-inserts a key of an earlier batch (a uniformly
    drawn earlier slot), so that about that fraction of the resident
    elements are replaced duplicates when the build ends; the cleanup
    measurements of sec. V-E remove 10 % and 50 %.  Followed by nq lookups
    of which half hit (keys drawn from the build).  Streams: 1 keys, 2
    values, 3 re-insert choice, 4 earlier slot, 6 lookups."""
    keys = uniform_keys(config, 1, 0, R * b).reshape(R, b)
    vals = values(config, 2, 0, R * b).reshape(R, b)
    flat = keys.reshape(-1)
    u = splitmix64(config, 3, 0, R * b).reshape(R, b)
    thresh = np.uint64(min(int(stale * 2.0**64), 2**64 - 1))
    for i in range(1, R):
        pick = np.nonzero(u[i] < thresh)[0]
        if pick.size:
            src = bounded(config, 4, i * b, pick.size, i * b)
            keys[i, pick] = flat[src]
    hit = flat[bounded(config, 6, 0, nq, R * b)]
    miss = uniform_keys(config, 6, 1 << 40, nq)
    half = bounded(config, 6, 1 << 41, nq, 2).astype(bool)
    look = np.where(half, hit, miss).astype(np.uint32)
    return PlainWorkload(name="cleanup b=%d R=%d stale=%.2f" % (b, R, stale), b=b, keys=keys,
                         vals=vals, is_delete=np.zeros(R, bool), lookups=look,
                         count_lo=np.zeros(0, np.uint32), count_hi=np.zeros(0, np.uint32),
                         range_lo=np.zeros(0, np.uint32), range_hi=np.zeros(0, np.uint32),
                         width=0, meta={"stale_target": stale})


def batching_stream(config: int = 4, n_batches: int = 4096, median: int = 4096,
                    sigma: float = 1.0, lo: int = 256, hi: int = 65536, b: int = 1 << 16):
    """User batches for the batching form: sizes round(exp(N(ln median,
    sigma))) clipped to [lo, min(hi, b)], uniform 31-bit keys; batch i
    deletes iff i mod 10 == 9, with keys drawn from earlier inserted keys.
    Returns a list of (keys, vals, is_delete).  Normal deviates come from
    the Box-Muller transform of two splitmix64 uniforms."""
    u1 = (splitmix64(config, 8, 0, n_batches) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (splitmix64(config, 9, 0, n_batches) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    sizes = np.clip(np.round(np.exp(np.log(median) + sigma * z)), lo, min(hi, b)).astype(np.int64)
    total = int(sizes.sum())
    keys = uniform_keys(config, 1, 0, total)
    vals = values(config, 2, 0, total)
    out = []
    off = 0
    ins_start, ins_cum = [], [0]  # inserted ranges, cumulative lengths
    draw = 0
    for i in range(n_batches):
        n = int(sizes[i])
        k = keys[off:off + n].copy()
        v = vals[off:off + n]
        dele = (i % 10) == 9
        if dele:
            idx = bounded(config, 3, draw, n, ins_cum[-1])
            draw += n
            cum = np.asarray(ins_cum, dtype=np.int64)
            which = np.searchsorted(cum, idx, side="right") - 1
            k = keys[np.asarray(ins_start, dtype=np.int64)[which] + (idx - cum[which])]
        else:
            ins_start.append(off)
            ins_cum.append(ins_cum[-1] + n)
        out.append((k, v, dele))
        off += n
    return out


# ---------------------------------------------------------------- serving
SERVING_KINDS = ("lookup", "count", "range", "insert", "delete")
SERVING_MIX = (0.50, 0.10, 0.10, 0.25, 0.05)


@dataclass
class ServingRequests:
    """Arrival-ordered requests.  Request r has kind[r] (index into
    SERVING_KINDS), size[r] operations and arrives at t_arrive[r] seconds.
    Payloads are laid out per kind in arrival order, so the requests of one
    kind admitted together form one contiguous slice: lookup_keys,
    count_lo/hi, range_lo/hi; inserts and deletes share one update stream of
    keys, values and delete flags (1 for a delete).  off[r] is the
    request's first element in its kind's stream."""
    t_arrive: np.ndarray
    kind: np.ndarray
    size: np.ndarray
    off: np.ndarray
    lookup_keys: np.ndarray
    count_lo: np.ndarray
    count_hi: np.ndarray
    range_lo: np.ndarray
    range_hi: np.ndarray
    upd_keys: np.ndarray
    upd_val: np.ndarray
    upd_is_del: np.ndarray
    width: int

    @property
    def n(self) -> int:
        return int(self.kind.size)


def resident(config: int = 5, b: int = 1 << 16, R: int = 4096):
    """The resident dictionary: R insert batches of b uniform 31-bit keys."""
    return (uniform_keys(config, 1, 0, R * b).reshape(R, b),
            values(config, 2, 0, R * b).reshape(R, b))


def serving_requests(resident_keys: np.ndarray, n_requests: int, rate: float, config: int = 5,
                     max_size: int = 8192, expected_hits: int = 32,
                     mix=SERVING_MIX) -> ServingRequests:
    """Poisson arrivals at `rate` requests/s; kinds drawn with probabilities
    `mix`; sizes log-uniform in [1, max_size]; lookups half drawn from the
    resident keys; count/range width so about `expected_hits` resident keys
    fall inside; inserts of fresh uniform keys; deletes of resident keys."""
    u = (splitmix64(config, 20, 0, n_requests) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    t = np.cumsum(-np.log1p(-u) / rate)
    c = (splitmix64(config, 21, 0, n_requests) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    kind = np.searchsorted(np.cumsum(mix), c, side="right").clip(0, len(mix) - 1).astype(np.uint8)
    s = (splitmix64(config, 22, 0, n_requests) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    size = np.clip(np.floor(np.exp(s * np.log(max_size + 1))), 1, max_size).astype(np.int64)
    off = np.zeros(n_requests, np.int64)
    res = resident_keys.reshape(-1)
    width = max(1, int(round(expected_hits * KEY_DOMAIN / res.size)))
    totals = []
    for k in range(len(SERVING_KINDS)):
        sel = kind == k
        if k == 4:  # deletes share the update stream with inserts
            continue
        off[sel] = np.concatenate([[0], np.cumsum(size[sel])[:-1]]) if sel.any() else 0
        totals.append(int(size[sel].sum()))
    upd = (kind == 3) | (kind == 4)
    off[upd] = np.concatenate([[0], np.cumsum(size[upd])[:-1]]) if upd.any() else 0
    n_lk, n_ct, n_rg = totals[0], totals[1], totals[2]
    pick = splitmix64(config, 23, 0, n_lk)
    hit = (pick & np.uint64(1)).astype(bool)
    idx = ((pick >> np.uint64(32)) * np.uint64(res.size)) >> np.uint64(32)
    lookup_keys = np.where(hit, res[idx.astype(np.int64)], uniform_keys(config, 24, 0, n_lk))
    starts = bounded(config, 25, 0, n_ct + n_rg, KEY_DOMAIN - width + 1).astype(np.uint32)
    n_upd = int(size[upd].sum())
    ins_keys = uniform_keys(config, 26, 0, n_upd)
    del_pick = bounded(config, 27, 0, n_upd, res.size)
    upd_is_del = np.repeat(kind[upd] == 4, size[upd])
    upd_keys = np.where(upd_is_del, res[del_pick], ins_keys).astype(np.uint32)
    upd_val = values(config, 28, 0, n_upd)
    return ServingRequests(t, kind, size, off, lookup_keys.astype(np.uint32),
                           starts[:n_ct], starts[:n_ct] + np.uint32(width - 1),
                           starts[n_ct:], starts[n_ct:] + np.uint32(width - 1),
                           upd_keys, upd_val, upd_is_del.astype(np.uint8), width)


def batching_queries(user_batches, config: int = 4, nq: int = 1 << 20, ncount: int = 1 << 16,
                     expected_hits: int = 16):
    """Queries for the batching form's user batches: query_set over the
    concatenated operations, each user batch its own batch number."""
    sizes = [u[0].size for u in user_batches]
    flat = np.concatenate([u[0] for u in user_batches])
    bidx = np.repeat(np.arange(len(user_batches)), sizes)
    dele = np.repeat(np.array([bool(u[2]) for u in user_batches]), sizes)
    return query_set(config, flat, bidx, dele, nq, ncount, expected_hits)
