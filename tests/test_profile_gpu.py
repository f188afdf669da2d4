"""GPU tests of the library's per-launch profiler (lsm_profile_*): launch
counts per kernel kind follow the path taken (the sort path's kernels, one
merge per full level the cascade passes, as the binary counter fixes), the
times are positive, and profiling changes no result."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd.lsm import KERNEL_NAMES, LSM
from _gpu import Trio, dev, ffz, host, note, pipeline_schedule

pytestmark = pytest.mark.gpu

K = {n: i for i, n in enumerate(KERNEL_NAMES)}


def default_fusion(b):
    j = 0
    while j < 8 and (b << (j + 1)) <= (1 << 20):
        j += 1
    return j


@pytest.mark.parametrize("mode,fusion,group", [
    (LSM.SORT_TOP_DIGIT, -1, 4), (LSM.SORT_TOP_DIGIT, 0, 4), (LSM.SORT_TOP_DIGIT, 2, 4),
    (LSM.SORT_TOP_DIGIT, 1, 4), (LSM.SORT_TOP_DIGIT, 0, 2), (LSM.SORT_TOP_DIGIT, 0, 1),
    (LSM.SORT_TOP_DIGIT, 2, 1), (LSM.SORT_DIGIT_PASSES, -1, 4),
])
def test_profile_counts_follow_the_path(mode, fusion, group):
    """Merge launches: one per level the cascade passes beyond the levels
    fused into the top-digit sort (none fused on the digit-pass path; the
    sort of a group of G batches takes the merges of the levels below
    log2 G, fused or not)."""
    b, R = 4096, 13
    rng = np.random.default_rng(5)
    note("profile counts mode=%d fusion=%d group=%d" % (mode, fusion, group))
    t = Trio(b)
    t.g.set_sort_path(mode)
    t.g.set_fusion(fusion)
    t.g.set_grouping(group)
    depth = 0 if mode == LSM.SORT_DIGIT_PASSES else (default_fusion(b) if fusion < 0 else fusion)
    t.g.profile(True)
    t.g.profile_read(reset=True)
    for _ in range(R):
        t.insert(rng.integers(0, 1 << 31, b, dtype=np.uint64).astype(np.uint32),
                 rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
    q = rng.integers(0, 1 << 31, 1000, dtype=np.uint64).astype(np.uint32)
    lo, hi = q[:300], q[:300] + 10**6
    gv, gf = t.g.lookup(dev(q))
    gc = t.g.count(dev(lo), dev(hi))
    go, gk, gval = t.g.range(dev(lo), dev(hi), cap=1 << 20)  # one lsm_range call
    torch.cuda.synchronize()
    ov, of = t.m.lookup(q)
    assert np.array_equal(host(gv), ov) and np.array_equal(host(gf), of)
    assert np.array_equal(host(gc), t.m.count(lo, hi))
    oo, ok, oval = t.m.range(lo, hi)
    assert np.array_equal(host(go), oo) and np.array_equal(host(gk), ok)
    assert np.array_equal(host(gval), oval)
    t.check_order(q[:200])
    p = t.g.profile_read(reset=True)
    t.g.profile(False)
    passes = 4  # 31-bit keys, status bit not sorted
    scat, step, lone, sorts = pipeline_schedule(R, group)
    if mode != LSM.SORT_TOP_DIGIT:
        sorts = [(r, 1) for r in range(R)]
    merges = sum(max(0, ffz(r) - max(depth, g.bit_length() - 1)) for r, g in sorts)
    expect = {"k_merge": merges, "k_lookup": 1, "k_order": 2,
              "k_range_emit": 1, "k_scan": 1, "k_count": 2}
    if mode == LSM.SORT_TOP_DIGIT:
        # Pipelined: scatters alone (the first batch's, and each batch that
        # joins a group), steps (a batch's scatter with the buckets of the
        # batch or group before it), and the buckets of what is pending when
        # the first query needs the levels.
        expect.update({"k_msd_scatter": scat, "k_sort_step": step, "k_local_sort": lone})
    else:
        expect.update({"k_sort_hist": R, "k_sort_pass": R * passes})
    for name, n in expect.items():
        assert int(p.launches[K[name]]) == n, (name, int(p.launches[K[name]]), n)
        assert n == 0 or p.kernel_ms[K[name]] > 0.0, name
    others = set(KERNEL_NAMES) - set(expect)
    assert all(int(p.launches[K[n]]) == 0 for n in others), [n for n in others if p.launches[K[n]]]
    assert p.update_calls == R and p.update_p50_ms > 0.0
    t.check_levels()


def test_profile_off_and_on_give_the_same_levels():
    b = 3000
    rng = np.random.default_rng(6)
    note("profile on/off equality")
    keys = [rng.integers(0, 5000, b).astype(np.uint32) for _ in range(9)]
    vals = [rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32) for _ in range(9)]
    out = []
    for prof in (False, True):
        g = LSM(b)
        g.profile(prof)
        for k, v in zip(keys, vals):
            g.insert(dev(k), dev(v))
        g.sync()
        out.append([tuple(host(x).tobytes() for x in g.level(i)) for i in g.occupied()])
        if prof:
            g.profile_read(reset=True)
        g.close()
    assert out[0] == out[1]
