"""GPU parity of the pipelined insertion: a batch sorted by the top-digit
sort has its tiles scattered by its own update call and its buckets sorted
(with the fused cascade) by the next call's launch or when anything reads
the levels.  Streams of many batches with no read in between run the
combined kernel on every call; the levels then equal the cascade oracle's
byte for byte and the answers the map oracle's.  Covers partial batches,
deletions, mixed batches, b across tile edges, fused depths, sort-path
switches in the middle of a stream (the digit-pass sort completes the
pending batch first), lsm_clear with a pending batch, the profile of the
pipeline, and pairs (a batch that would fill level 0 waits for the next
one; both are sorted together into the level the second fills).  Integer
results, tolerance 0."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import KERNEL_NAMES, LSM, LSMError, LSM_EINVAL
from _gpu import Trio, dev, dev_u8, host, note, pipeline_schedule

pytestmark = pytest.mark.gpu

K = {n: i for i, n in enumerate(KERNEL_NAMES)}


def feed(t, ops, rng=None, mixed_every=0):
    for i, (kind, k, v) in enumerate(ops):
        if mixed_every and i % mixed_every == mixed_every - 1:
            vv = v if v is not None else k
            t.mixed(k, vv, (rng.random(k.size) < 0.4).astype(np.uint8))
        elif kind == "insert":
            t.insert(k, v)
        else:
            t.delete(k)


@pytest.mark.parametrize("b,R,domain", [(1, 70, 9), (64, 67, 3000), (2047, 33, 5000),
                                        (4099, 40, 1 << 14), (10000, 35, 1 << 31),
                                        (1 << 16, 35, 1 << 31)])
def test_unread_stream_equals_oracle(b, R, domain):
    """Every batch through the pipeline (the top-digit path is forced: keys
    below 2^14 put a whole batch into one top-digit bucket, which would move
    the automatic choice to digit passes from b = 4099 on; such a bucket is
    sorted by the streaming fallback inside the pipeline instead)."""
    note("pipelined stream b=%d R=%d" % (b, R))
    ops, q, lo, hi = W.random_small(900 + b, b, R, domain, p_delete=0.3, nq=500)
    t = Trio(b)
    t.g.set_sort_path(LSM.SORT_TOP_DIGIT)
    feed(t, ops, np.random.default_rng(b), mixed_every=7)
    t.check_levels()
    t.check_queries(q, lo, hi)
    st = t.g.stats()
    assert st.sorts_top_digit == R and st.sorts_digit_passes == 0
    t.g.close()


def test_path_switches_and_fusion_changes_mid_stream():
    """Forced sort-path and fusion changes between batches: a digit-pass
    batch completes the pending top-digit one first."""
    b, R = 3000, 40
    note("pipeline path switches b=%d" % b)
    ops, q, lo, hi = W.random_small(77, b, R, 1 << 20, p_delete=0.25, nq=400)
    t = Trio(b)
    modes = [LSM.SORT_AUTO, LSM.SORT_DIGIT_PASSES, LSM.SORT_TOP_DIGIT]
    for i, (kind, k, v) in enumerate(ops):
        t.g.set_sort_path(modes[(i // 3) % 3])
        t.g.set_fusion([-1, 0, 2, 5][(i // 5) % 4])
        if kind == "insert":
            t.insert(k, v)
        else:
            t.delete(k)
        if i % 11 == 10:
            t.check_queries(q, lo, hi)
    t.check_levels()
    t.check_queries(q, lo, hi)
    st = t.g.stats()
    assert st.sorts_top_digit + st.sorts_digit_passes == R
    assert st.sorts_top_digit > 0 and st.sorts_digit_passes > 0
    t.g.close()


def test_clear_drops_the_pending_batch():
    b = 512
    note("pipeline clear b=%d" % b)
    rng = np.random.default_rng(3)
    t = Trio(b)
    for _ in range(5):
        k = rng.integers(0, 10**6, b).astype(np.uint32)
        t.g.insert(dev(k), dev(k))  # pending at the end; never read
    t.g.clear()
    assert t.g.num_batches == 0
    ops, q, lo, hi = W.random_small(5, b, 9, 4000, nq=300)
    feed(t, ops)
    t.check_levels()
    t.check_queries(q, lo, hi)
    t.g.close()


@pytest.mark.parametrize("group,R", [(1, 21), (2, 21), (2, 20), (4, 21), (4, 22), (4, 23)])
def test_pipeline_profile_and_sync(group, R):
    """R batches with no read between them, then lsm_sync.  Without
    grouping: one scatter, R - 1 steps, and lsm_sync completes the last batch
    (one bucket sort).  With groups of G, a batch whose counter is a multiple
    of G waits for the next G - 1 (their scatters run alone), the group's
    bucket sort runs beside the next group's first scatter, and lsm_sync
    sorts what is pending (an incomplete group as groups of 2 and 1).  The
    levels are then complete."""
    b = 4096
    note("pipeline profile b=%d R=%d group=%d" % (b, R, group))
    rng = np.random.default_rng(8)
    t = Trio(b)
    t.g.set_sort_path(LSM.SORT_TOP_DIGIT)
    t.g.set_grouping(group)
    t.g.profile(True)
    t.g.profile_read(reset=True)
    for _ in range(R):
        t.insert(rng.integers(0, 1 << 31, b, dtype=np.uint64).astype(np.uint32),
                 rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32))
    t.g.sync()
    p = t.g.profile_read(reset=True)
    scat, step, lone, sorts = pipeline_schedule(R, group)
    # Closed forms of the schedule (the helper is checked against them).
    if group == 1:
        assert (scat, step, lone) == (1, R - 1, 1)
    else:
        full = (R - 1) // group  # complete groups followed by a later batch
        assert (scat, step, lone) == (R - full, full, bin(R - full * group).count("1"))
    assert sum(g for _, g in sorts) == R
    assert int(p.launches[K["k_msd_scatter"]]) == scat
    assert int(p.launches[K["k_sort_step"]]) == step
    assert int(p.launches[K["k_local_sort"]]) == lone
    assert p.update_calls == R
    t.g.profile(False)
    t.check_levels()
    t.g.close()


@pytest.mark.parametrize("b,domain,group", [
    (1, 1 << 31, 4), (2048, 1 << 31, 4), (2049, 1 << 31, 4), (30000, 1 << 31, 4),
    (256, 779, 4), (700, 1500, 2), (3000, 9000, 4), (1 << 17, 1 << 31, 4),
    ((1 << 17) + 1, 1 << 31, 4), ((1 << 18) + 1, 1 << 31, 4)])
def test_grouping_gives_the_same_levels(b, domain, group):
    """The same stream (partial, deleting and mixed batches) with grouping
    on and off: the levels equal the cascade oracle's and each other byte
    for byte.  The grouped dictionary is read at random points (a read
    completes an incomplete group, so groups of 1, 2 and 4 all occur).
    Small key domains put every key into one top-digit bucket, so a group's
    bucket is ranked by the LDS radix passes (<= 1536 elements) or in global
    memory, and keys repeat across the batches of a group and within mixed
    batches.  b = 2^17 is the largest batch for groups of four (all tiles in
    one group table), 2^17 + 1 takes pairs, 2^18 + 1 no groups."""
    R = 13 if b >= 1 << 17 else 37
    note("grouping on/off b=%d domain=%d group=%d R=%d" % (b, domain, group, R))
    ops, q, lo, _ = W.random_small(4400 + b % 97, b, R, domain, p_delete=0.3, nq=300)
    # Ranges of about 40 keys at the largest sizes (the map oracle lists every pair).
    hi = np.minimum(lo.astype(np.int64) + max(40 * domain // (b * R), 8), 2**32 - 1).astype(np.uint32)
    rng = np.random.default_rng(b)
    reads = set(rng.choice(R, size=R // 5, replace=False).tolist())
    tr = [Trio(b), Trio(b)]
    tr[0].g.set_grouping(group)
    tr[1].g.set_grouping(1)
    for t in tr:
        t.g.set_sort_path(LSM.SORT_TOP_DIGIT)
    for i, (kind, k, v) in enumerate(ops):
        dl = (rng.random(k.size) < 0.5).astype(np.uint8)
        for t in tr:
            if kind == "insert":
                t.insert(k, v)
            elif i % 4 == 3:
                t.mixed(k, k, dl)
            else:
                t.delete(k)
        if i in reads:
            tr[0].check_queries(q[:50], lo[:20], hi[:20])
    for t in tr:
        t.check_levels()
    for i in tr[0].c.occupied():
        a, c = tr[0].g.level(i), tr[1].g.level(i)
        assert all(np.array_equal(host(x), host(y)) for x, y in zip(a, c)), i
    tr[0].check_queries(q, lo, hi)
    st = tr[0].g.stats()
    assert st.sorts_top_digit == R
    for t in tr:
        t.g.close()


def test_mixed_batches_never_group():
    """Mixed batches sort a key's tombstone before its insertion; across the
    batches of a group that would put an older tombstone before a newer
    insertion, so they never join a group: a stream of mixed batches over a
    small key domain (keys repeating within and across batches) runs one
    scatter and then steps only, and its levels equal the cascade oracle's."""
    b, R = 256, 24
    note("mixed batches never group b=%d" % b)
    rng = np.random.default_rng(11)
    t = Trio(b)
    t.g.set_sort_path(LSM.SORT_TOP_DIGIT)
    t.g.profile(True)
    t.g.profile_read(reset=True)
    for _ in range(R):
        k = rng.integers(0, 600, b).astype(np.uint32)
        t.mixed(k, rng.integers(0, 2**32, b, dtype=np.uint64).astype(np.uint32),
                (rng.random(b) < 0.5).astype(np.uint8))
    t.g.sync()
    p = t.g.profile_read(reset=True)
    t.g.profile(False)
    scat, step, lone, _ = pipeline_schedule(R, group=1)
    assert int(p.launches[K["k_msd_scatter"]]) == scat
    assert int(p.launches[K["k_sort_step"]]) == step
    assert int(p.launches[K["k_local_sort"]]) == lone
    t.check_levels()
    q = np.arange(602, dtype=np.uint32)
    t.check_queries(q, q[:300:3], q[:300:3] + 40)
    t.g.close()


@pytest.mark.parametrize("b,asked,effective", [(4096, 0, 1), (4096, 3, 2), (4096, 100, 4),
                                               (1 << 18, 4, 2), ((1 << 18) + 1, 2, 1)])
def test_grouping_argument_is_rounded_and_capped(b, asked, effective):
    """lsm_set_grouping rounds down to 1, 2 or 4 and caps by b (four when
    4 tiles of every batch fit one group table, two for b <= 2^18): the
    launch schedule of 9 unread batches is that of the effective size."""
    note("grouping argument b=%d asked=%d" % (b, asked))
    R = 9
    rng = np.random.default_rng(b + asked)
    g = LSM(b)
    g.set_sort_path(LSM.SORT_TOP_DIGIT)
    g.set_grouping(asked)
    g.profile(True)
    g.profile_read(reset=True)
    for _ in range(R):
        k = rng.integers(0, 1 << 31, b, dtype=np.uint64).astype(np.uint32)
        g.insert(dev(k), dev(k))
    g.sync()
    p = g.profile_read(reset=True)
    scat, step, lone, _ = pipeline_schedule(R, effective)
    assert (int(p.launches[K["k_msd_scatter"]]), int(p.launches[K["k_sort_step"]]),
            int(p.launches[K["k_local_sort"]])) == (scat, step, lone)
    with pytest.raises(LSMError) as ei:
        g.set_grouping(-1)
    assert ei.value.status == LSM_EINVAL
    g.close()


@pytest.mark.parametrize("depth", [0, 1, 16])
def test_pacing_depth_changes_nothing(depth):
    """Launch pacing only delays the host: free-running (0), one launch
    ahead (1) or sixteen ahead, the same unread stream of full, partial,
    deleting and mixed batches gives the cascade oracle's levels byte for
    byte and the map oracle's answers.  A negative depth is refused."""
    b, R = 5000, 37
    note("pacing depth %d" % depth)
    ops, q, lo, hi = W.random_small(7100 + depth, b, R, 1 << 31, p_delete=0.3, nq=200)
    t = Trio(b)
    t.g.set_sort_path(LSM.SORT_TOP_DIGIT)
    t.g.set_max_inflight(depth)
    feed(t, ops, np.random.default_rng(depth), mixed_every=5)
    t.check_levels()
    t.check_queries(q, lo, hi)
    with pytest.raises(LSMError) as ei:
        t.g.set_max_inflight(-1)
    assert ei.value.status == LSM_EINVAL
    t.g.close()
