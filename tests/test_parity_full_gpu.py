"""Parity at the paper-scale size the benchmark times (b = 2^16, 1024 update
batches, n = 2^26 slots), in the benchmark's launch configuration.

* The one occupied level (level 10, 2^26 elements) is compared byte for byte
  with the cascade oracle.
* Sampled lookups / counts / ranges are compared with the map oracle.  The
  oracle replays, in batch order, exactly the operations whose keys can
  affect the sampled queries (a dictionary's answer for a key depends only
  on that key's own operations), so it answers those queries exactly
  without holding all 2^26 operations.
* Properties that hold at any size are checked on every query: count equals
  the range size, range keys ascend within their bounds, and each returned
  pair is what lookup returns for its key.
* Cleanup at full size: the cascade oracle's cleanup gives the live set in
  key order, which fixes every successor / predecessor answer exactly; the
  GPU answers all 2^22 order queries before and after its own cleanup, and
  its cleaned levels equal the oracle's byte for byte.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import LSM
from _gpu import dev, host, note

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _filtered_map(w, keep):
    """Map oracle fed, in batch order, the operations whose key passes keep()."""
    m = oracle.MapOracle()
    for i in range(w.R):
        k = w.keys[i]
        sel = keep(k)
        if not sel.any():
            continue
        if w.is_delete[i]:
            m.delete(k[sel])
        else:
            m.insert(k[sel], w.vals[i][sel])
    return m


def _in_intervals(lo, hi):
    order = np.argsort(lo, kind="stable")
    slo, shi = lo[order].astype(np.int64), hi[order].astype(np.int64)
    run_hi = np.maximum.accumulate(shi)

    def keep(k):
        k = k.astype(np.int64)
        j = np.searchsorted(slo, k, side="right") - 1
        ok = j >= 0
        return ok & (k <= run_hi[np.maximum(j, 0)])
    return keep


def test_paper_scale_layout_and_sampled_queries():
    w = W.paper_scale()
    note("paper scale b=2^16 R=1024: GPU build")
    g = LSM(w.b)
    keys_d, vals_d = dev(w.keys), dev(w.vals)
    for i in range(w.R):
        if w.is_delete[i]:
            g.delete(keys_d[i])
        else:
            g.insert(keys_d[i], vals_d[i])
    torch.cuda.synchronize()
    assert g.num_batches == 1024 and g.occupied() == [10]

    note("paper scale: cascade oracle")
    c = oracle.CascadeOracle(w.b)
    for i in range(w.R):
        if w.is_delete[i]:
            c.delete(w.keys[i])
        else:
            c.insert(w.keys[i], w.vals[i])
    okv, ov = c.level(10)
    gkv, gv = g.level(10)
    gkv, gv = host(gkv), host(gv)
    assert np.array_equal(gkv, okv), "level 10 key variables differ"
    assert np.array_equal(gv, ov), "level 10 values differ"
    del okv, ov, gkv, gv
    n_valid = c.cleanup()
    cleaned = {i: c.level(i) for i in c.occupied()}
    r_clean = c.r
    del c

    note("paper scale: queries")
    q_d = dev(w.lookups)
    lv, lf = g.lookup(q_d)
    cnt = g.count(dev(w.count_lo), dev(w.count_hi))
    rcnt = g.count(dev(w.range_lo), dev(w.range_hi))
    roff, rk, rv = g.range(dev(w.range_lo), dev(w.range_hi))
    torch.cuda.synchronize()
    lv, lf, cnt, rcnt = host(lv), host(lf), host(cnt), host(rcnt)
    roff, rk, rv = host(roff).astype(np.int64), host(rk), host(rv)

    # Properties at full size, every query.
    assert np.array_equal(np.diff(roff), rcnt.astype(np.int64)), "count != range size"
    qid = np.repeat(np.arange(w.range_lo.size), np.diff(roff))
    assert np.all(rk >= w.range_lo[qid]) and np.all(rk <= w.range_hi[qid])
    same_q = qid[1:] == qid[:-1]
    assert np.all(rk[1:][same_q] > rk[:-1][same_q]), "range keys not strictly ascending"
    samp = np.linspace(0, rk.size - 1, 50000).astype(np.int64)
    sv, sf = g.lookup(dev(rk[samp]))
    torch.cuda.synchronize()
    assert np.all(host(sf) == 1) and np.array_equal(host(sv), rv[samp])
    assert 0.40 < lf.mean() < 0.55

    # Sampled queries against the map oracle.
    qi = np.linspace(0, w.lookups.size - 1, 20000).astype(np.int64)
    qs = np.unique(w.lookups[qi])
    m = _filtered_map(w, lambda k: np.isin(k, qs))
    ov, of = m.lookup(w.lookups[qi])
    assert np.array_equal(lf[qi], of) and np.array_equal(lv[qi], ov)

    ci = np.linspace(0, w.count_lo.size - 1, 3000).astype(np.int64)
    m = _filtered_map(w, _in_intervals(w.count_lo[ci], w.count_hi[ci]))
    assert np.array_equal(cnt[ci], m.count(w.count_lo[ci], w.count_hi[ci]))

    ri = np.linspace(0, w.range_lo.size - 1, 3000).astype(np.int64)
    m = _filtered_map(w, _in_intervals(w.range_lo[ri], w.range_hi[ri]))
    oo, ok, oval = m.range(w.range_lo[ri], w.range_hi[ri])
    got_k = np.concatenate([rk[roff[j]:roff[j + 1]] for j in ri])
    got_v = np.concatenate([rv[roff[j]:roff[j + 1]] for j in ri])
    assert np.array_equal(np.diff(oo.astype(np.int64)), np.diff(roff)[ri])
    assert np.array_equal(got_k, ok) and np.array_equal(got_v, oval)

    # Order queries, exact for every query: the oracle's cleaned list is the
    # live set in key order.
    note("paper scale: order queries and cleanup")
    flat_kv = np.concatenate([cleaned[i][0] for i in sorted(cleaned)])
    flat_v = np.concatenate([cleaned[i][1] for i in sorted(cleaned)])
    live_k, live_v = (flat_kv[:n_valid] >> 1).astype(np.int64), flat_v[:n_valid]
    assert np.all(flat_kv[:n_valid] & 1 == 1) and np.all(np.diff(live_k) > 0)
    edges = np.array([0, 1, 2**31 - 2, 2**31 - 1, 2**31, 2**32 - 1], np.uint32)
    q = np.concatenate([w.lookups, edges, (live_k[::4099] + 1).astype(np.uint32)])
    qi = q.astype(np.int64)
    js = np.searchsorted(live_k, qi, side="right")
    jp = np.searchsorted(live_k, qi, side="left") - 1
    exp = {"successor": (js < n_valid, np.minimum(js, n_valid - 1)),
           "predecessor": (jp >= 0, np.maximum(jp, 0))}

    def check_order(stage):
        for name, (f, j) in exp.items():
            gk, gv2, gf = getattr(g, name)(dev(q))
            torch.cuda.synchronize()
            gk, gv2, gf = host(gk), host(gv2), host(gf)
            assert np.array_equal(gf, f.astype(np.uint8)), "%s found flags differ (%s)" % (name, stage)
            assert np.array_equal(gk, np.where(f, live_k[j], 0).astype(np.uint32)), \
                "%s keys differ (%s)" % (name, stage)
            assert np.array_equal(gv2, np.where(f, live_v[j], 0).astype(np.uint32)), \
                "%s values differ (%s)" % (name, stage)

    check_order("before cleanup")
    assert g.cleanup() == n_valid
    g.sync()
    assert g.num_batches == r_clean and g.occupied() == sorted(cleaned)
    for i, (okv, ov) in cleaned.items():
        gkv, gv = g.level(i)
        assert np.array_equal(host(gkv), okv), "cleaned level %d key variables differ" % i
        assert np.array_equal(host(gv), ov), "cleaned level %d values differ" % i
    check_order("after cleanup")
    lv2, lf2 = g.lookup(q_d)
    torch.cuda.synchronize()
    assert np.array_equal(host(lf2), lf) and np.array_equal(host(lv2), lv)
    g.close()
