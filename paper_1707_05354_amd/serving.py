"""Serving form: continuous batching of mixed dictionary requests over a GPU
LSM kept resident on the device.

Requests are single-type (lookup, count, range, insert, delete) and arrive
over time.  The loop forms epochs (the batch semantics of sec. III-A:
queries and updates run in separate phases):

  1. admit, in arrival order, every request that has arrived, up to an
     operation budget per epoch and while the range results' worst-case size
     fits the free part of a result pool sized from free HBM;
  2. enqueue the epoch's queries against the state left by earlier epochs:
     one lsm_lookup, one lsm_count and one lsm_range_async over the epoch's
     contiguous slices (each kind's payloads are laid out in arrival order);
  3. enqueue the epoch's updates, in arrival order, through the coalescer
     (lsm_submit_mixed: keys, values and delete flags, encoded by the
     library) and flush, so the next epoch sees them.

Epochs are enqueued without waiting for earlier ones (up to `in_flight`
epochs on the device), so requests that arrive while an epoch runs are
admitted into the next one and their work is queued behind it on the
device.  A request completes when its epoch's completion event fires; its
latency is that time minus its arrival time.

Every step runs in the library's HIP kernels; this module only decides what
to admit and slices device arrays.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import lsm as L
from .workload import ServingRequests

LOOKUP, COUNT, RANGE, INSERT, DELETE = range(5)


def plan_epoch(t_arrive: np.ndarray, size: np.ndarray, range_cost: np.ndarray, i: int,
               now: float, max_ops: int, range_room: int) -> int:
    """End (exclusive) of the epoch that starts at request i: requests that
    arrived by `now`, in arrival order, while the epoch's operations stay
    within max_ops and its worst-case range output within range_room.  At
    least one arrived request is admitted when its range cost fits at all;
    returns i when nothing can be admitted."""
    arrived = int(np.searchsorted(t_arrive, now, side="right"))
    if arrived <= i:
        return i
    ops = np.cumsum(size[i:arrived])
    rc = np.cumsum(range_cost[i:arrived])
    ok = (ops <= max_ops) & (rc <= range_room)
    n = int(np.argmin(ok)) if not ok.all() else ok.size
    if n == 0 and range_cost[i] <= range_room:
        n = 1  # one request larger than the operation budget runs alone
    return i + n


class RangePool:
    """Ring of range-result slots in one device buffer.  Every epoch takes
    one slot (possibly empty) sized for the worst case of its range output;
    slots are released in epoch order once their epoch has completed."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.slots = []          # (start, length), oldest first
        self.head = 0            # end of the newest non-empty slot

    def _tail(self):
        for start, n in self.slots:
            if n > 0:
                return start
        return None

    def room(self) -> int:
        """Largest slot that reserve() can hand out right now."""
        tail = self._tail()
        if tail is None:
            return self.capacity
        if self.head > tail:
            return max(self.capacity - self.head, tail)
        return tail - self.head

    def reserve(self, n: int) -> Optional[int]:
        n = int(n)
        tail = self._tail()
        if n == 0:
            start = self.head if tail is not None else 0
        elif tail is None:
            if n > self.capacity:
                return None
            start = 0
        elif self.head > tail:
            if self.capacity - self.head >= n:
                start = self.head
            elif tail >= n:
                start = 0
            else:
                return None
        else:
            if tail - self.head >= n:
                start = self.head
            else:
                return None
        self.slots.append((start, n))
        if n > 0:
            self.head = start + n
        elif tail is None:
            self.head = 0
        return start

    def release_oldest(self) -> None:
        self.slots.pop(0)


@dataclass
class Epoch:
    first: int
    last: int                     # exclusive
    event: torch.cuda.Event
    range_base: int = 0           # element offset of its range slot
    range_off_base: int = 0       # entry offset of its range offsets
    n_range_q: int = 0
    done_ms: float = float("nan")


@dataclass
class ServeResult:
    epochs: List[Epoch]
    latency_s: np.ndarray         # per request
    completion_s: np.ndarray      # per request, since the start
    wall_s: float
    ops: int
    stats: dict = field(default_factory=dict)


class Server:
    """Continuous-batching request loop over one LSM handle."""

    def __init__(self, g: "L.LSM", reqs: ServingRequests, max_epoch_ops: int = 1 << 20,
                 in_flight: int = 2, pool_elems: Optional[int] = None,
                 hbm_fraction: float = 0.25, keep_results: bool = False,
                 capture_ranges=False):
        self.g = g
        self.r = reqs
        self.max_epoch_ops = int(max_epoch_ops)
        self.in_flight = max(1, int(in_flight))
        dev = torch.device("cuda", g.device)

        def up(a, dtype=torch.int32):
            a = np.ascontiguousarray(a)
            if a.dtype == np.uint32:
                a = a.view(np.int32)
            return torch.from_numpy(a).to(dev)

        self.lk = up(reqs.lookup_keys)
        self.clo, self.chi = up(reqs.count_lo), up(reqs.count_hi)
        self.rlo, self.rhi = up(reqs.range_lo), up(reqs.range_hi)
        self.ukey, self.uval = up(reqs.upd_keys), up(reqs.upd_val)
        self.udel = up(reqs.upd_is_del, torch.uint8)
        self.lk_val = torch.empty(max(1, reqs.lookup_keys.size), dtype=torch.int32, device=dev)
        self.lk_found = torch.empty(max(1, reqs.lookup_keys.size), dtype=torch.uint8, device=dev)
        self.cnt = torch.empty(max(1, reqs.count_lo.size), dtype=torch.int32, device=dev)
        # Worst case of a range request's output: its queries' widths.
        w = (reqs.range_hi.astype(np.int64) - reqs.range_lo.astype(np.int64) + 1)
        self.range_cost = np.zeros(reqs.n, np.int64)
        rsel = reqs.kind == RANGE
        if rsel.any():
            starts = reqs.off[rsel]
            cw = np.concatenate([[0], np.cumsum(w)])
            self.range_cost[rsel] = cw[starts + reqs.size[rsel]] - cw[starts]
        # Range result pool from free HBM (admission by memory).
        free, _ = torch.cuda.mem_get_info(dev)
        if pool_elems is None:
            pool_elems = int(free * hbm_fraction) // 8
        if keep_results:
            pool_elems = max(pool_elems, int(self.range_cost.sum()))
        self.pool = RangePool(pool_elems)
        self.keep = keep_results
        # capture_ranges: each epoch's range output is copied to the host
        # when the epoch retires, before its result slot can be reused (True:
        # every epoch; a callable (first, last) -> bool: the epochs of
        # requests [first, last) it accepts).
        self.capture = capture_ranges
        self.captured = {}
        self.rk = torch.empty(max(1, pool_elems), dtype=torch.int32, device=dev)
        self.rv = torch.empty(max(1, pool_elems), dtype=torch.int32, device=dev)
        n_rq = int(reqs.range_lo.size)
        self.roff = torch.empty(n_rq + reqs.n + 1, dtype=torch.int64, device=dev)
        self._lib, self._h = g._lib, g._h

    # -- one epoch -----------------------------------------------------------
    def _enqueue(self, i: int, j: int, base: int, off_base: int) -> Epoch:
        r = self.r
        kinds = r.kind[i:j]
        lib, h = self._lib, self._h

        def span(k):
            sel = np.nonzero(kinds == k)[0]
            if sel.size == 0:
                return 0, 0
            a = int(r.off[i + sel[0]])
            e = int(r.off[i + sel[-1]] + r.size[i + sel[-1]])
            return a, e

        a, e = span(LOOKUP)
        if e > a:
            L._check(lib.lsm_lookup(h, self.lk.data_ptr() + 4 * a, e - a,
                                    self.lk_val.data_ptr() + 4 * a,
                                    self.lk_found.data_ptr() + a), "lsm_lookup")
        a, e = span(COUNT)
        if e > a:
            L._check(lib.lsm_count(h, self.clo.data_ptr() + 4 * a, self.chi.data_ptr() + 4 * a,
                                   e - a, self.cnt.data_ptr() + 4 * a), "lsm_count")
        a, e = span(RANGE)
        nrq = e - a
        if nrq > 0:
            cap = int(self.range_cost[i:j].sum())
            L._check(lib.lsm_range_async(h, self.rlo.data_ptr() + 4 * a, self.rhi.data_ptr() + 4 * a,
                                         nrq, self.roff.data_ptr() + 8 * off_base,
                                         self.rk.data_ptr() + 4 * base, self.rv.data_ptr() + 4 * base,
                                         cap), "lsm_range_async")
        upd = (kinds == INSERT) | (kinds == DELETE)
        if upd.any():
            sel = np.nonzero(upd)[0]
            ua = int(r.off[i + sel[0]])
            ue = int(r.off[i + sel[-1]] + r.size[i + sel[-1]])
            L._check(lib.lsm_submit_mixed(h, self.ukey.data_ptr() + 4 * ua,
                                          self.uval.data_ptr() + 4 * ua,
                                          self.udel.data_ptr() + ua, ue - ua),
                     "lsm_submit_mixed")
            L._check(lib.lsm_flush(h), "lsm_flush")
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        return Epoch(i, j, ev, base, off_base, nrq)

    # -- the loop ------------------------------------------------------------
    def run(self, realtime: bool = True) -> ServeResult:
        """Serve every request.  realtime=True follows the arrival clock;
        realtime=False treats all requests as arrived (epochs then depend
        only on the budgets)."""
        r = self.r
        t_arr = r.t_arrive if realtime else np.zeros_like(r.t_arrive)
        epochs: List[Epoch] = []
        pending: List[Epoch] = []
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i = 0
        off_base = 0
        while i < r.n:
            now = time.perf_counter() - t0
            if t_arr[i] > now:
                if pending and pending[0].event.query():
                    self._retire(pending)
                    continue
                if not pending:
                    time.sleep(min(1e-3, max(0.0, t_arr[i] - now)))
                continue
            room = self.pool.room()
            j = plan_epoch(t_arr, r.size, self.range_cost, i, now, self.max_epoch_ops, room)
            if j == i:  # result pool full: wait for the oldest epoch
                if not pending:
                    raise RuntimeError("a range request needs more result memory than the pool")
                pending[0].event.synchronize()
                self._retire(pending)
                continue
            cost = int(self.range_cost[i:j].sum())
            base = self.pool.reserve(cost)
            if base is None:
                pending[0].event.synchronize()
                self._retire(pending)
                continue
            ep = self._enqueue(i, j, base, off_base)
            off_base += ep.n_range_q + 1
            epochs.append(ep)
            pending.append(ep)
            i = j
            while len(pending) > self.in_flight:
                pending[0].event.synchronize()
                self._retire(pending)
        torch.cuda.synchronize()
        while pending:
            self._retire(pending)
        wall = time.perf_counter() - t0
        comp = np.empty(r.n)
        for ep in epochs:
            ep.done_ms = ref.elapsed_time(ep.event)
            comp[ep.first:ep.last] = ep.done_ms * 1e-3
        self.g.sync()
        lat = comp - t_arr
        return ServeResult(epochs, lat, comp, wall, int(r.size.sum()),
                           {"epochs": len(epochs), "pool_elems": self.pool.capacity})

    def _retire(self, pending: List[Epoch]) -> None:
        """Called once the oldest pending epoch has completed."""
        ep = pending.pop(0)
        want = self.capture(ep.first, ep.last) if callable(self.capture) else self.capture
        if want and ep.n_range_q:
            off = self.roff[ep.range_off_base: ep.range_off_base + ep.n_range_q + 1].cpu().numpy()
            n = int(off[-1])
            self.captured[ep.first] = (
                off, self.rk[ep.range_base: ep.range_base + n].cpu().numpy().view(np.uint32),
                self.rv[ep.range_base: ep.range_base + n].cpu().numpy().view(np.uint32))
        if not self.keep:
            self.pool.release_oldest()

    # -- results (after run) ---------------------------------------------------
    def results(self, res: ServeResult, req: int):
        """Host copy of one request's answer: (vals, found) for a lookup,
        counts for a count, (offsets, keys, vals) for a range (offsets
        relative to the request), None for an update."""
        r = self.r
        k, a, n = int(r.kind[req]), int(r.off[req]), int(r.size[req])
        if k == LOOKUP:
            return (self.lk_val[a:a + n].cpu().numpy().view(np.uint32),
                    self.lk_found[a:a + n].cpu().numpy())
        if k == COUNT:
            return self.cnt[a:a + n].cpu().numpy().view(np.uint32)
        if k == RANGE:
            ep = next(e for e in res.epochs if e.first <= req < e.last)
            kinds = r.kind[ep.first:ep.last]
            first_q = int(r.off[ep.first + np.nonzero(kinds == RANGE)[0][0]])
            qa = a - first_q
            if ep.first in self.captured:
                eo, ek, ev = self.captured[ep.first]
                off = eo[qa: qa + n + 1]
                s, e = int(off[0]), int(off[-1])
                return off - off[0], ek[s:e], ev[s:e]
            if not self.keep:
                raise RuntimeError("range results were released; serve with keep_results "
                                   "or capture_ranges")
            off = self.roff[ep.range_off_base + qa: ep.range_off_base + qa + n + 1].cpu().numpy()
            s, e = int(off[0]), int(off[-1])
            keys = self.rk[ep.range_base + s: ep.range_base + e].cpu().numpy().view(np.uint32)
            vals = self.rv[ep.range_base + s: ep.range_base + e].cpu().numpy().view(np.uint32)
            return off - off[0], keys, vals
        return None


def percentiles(lat: np.ndarray):
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}
