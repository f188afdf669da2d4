"""CPU tests of the serving loop's host logic: epoch admission and the
range-result pool (no GPU)."""
import numpy as np
import pytest

from paper_1707_05354_amd.serving import RangePool, plan_epoch


def test_plan_epoch_admits_arrived_requests_within_budgets():
    t = np.array([0.0, 0.1, 0.2, 0.3, 0.4])
    size = np.array([10, 20, 30, 40, 50])
    cost = np.array([0, 100, 0, 100, 0])
    assert plan_epoch(t, size, cost, 0, 0.25, 1000, 1000) == 3      # arrival
    assert plan_epoch(t, size, cost, 0, 1.0, 60, 1000) == 3         # op budget 10+20+30
    assert plan_epoch(t, size, cost, 0, 1.0, 1000, 150) == 3        # range budget
    assert plan_epoch(t, size, cost, 1, 1.0, 5, 1000) == 2          # one big request alone
    assert plan_epoch(t, size, cost, 1, 1.0, 1000, 50) == 1         # cannot fit: nothing
    assert plan_epoch(t, size, cost, 2, 0.15, 1000, 1000) == 2      # not arrived yet


def test_range_pool_never_overlaps_live_slots():
    """Random reservations and in-order releases against an occupancy
    model: live slots never overlap, stay inside the buffer, and room()
    is always a size that reserve() accepts."""
    rng = np.random.default_rng(0)
    for trial in range(200):
        cap = int(rng.integers(1, 200))
        pool = RangePool(cap)
        live = []
        for step in range(300):
            if live and rng.random() < 0.45:
                pool.release_oldest()
                live.pop(0)
                continue
            n = int(rng.integers(0, cap + 5)) if rng.random() < 0.9 else 0
            room = pool.room()
            start = pool.reserve(n)
            if start is None:
                assert n > room
                continue
            assert n <= room or n == 0
            assert 0 <= start and start + n <= cap
            live.append((start, n))
            occ = np.zeros(cap, int)
            for s, m in live:
                occ[s:s + m] += 1
            assert occ.max(initial=0) <= 1, (trial, step)
