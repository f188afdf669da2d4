"""Parity at the paper-scale size the benchmark times (b = 2^16, n = 2^26
slots, batch i deletes iff i mod 10 == 9), in the benchmark's launch
configuration, at two points of the build:

* r = 1023: levels 0..9 all full, the multi-level case of the paper's query
  tables.  Every level is compared byte for byte with the cascade oracle,
  then lookups, counts and ranges are run.
* r = 1024: the one occupied level (level 10, 2^26 elements) is compared
  byte for byte, and the same queries are run again.

Query answers: properties that hold at any size are checked on every query
(count equals the range size, range keys ascend within their bounds, each
returned pair is what lookup returns); a sample of every query kind is
compared with the map oracle fed only the operations on the sampled keys
(exact for those queries, see _fullsize).

Cleanup at full size: the cascade oracle's cleanup gives the live set in key
order, which fixes every successor / predecessor answer exactly; the GPU
answers all 2^22 order queries before and after its own cleanup, and its
cleaned levels equal the oracle's byte for byte.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import LSM, LSMError
from _fullsize import FilteredMap, check_range_properties, key_filter, ranges_of
from _gpu import dev, host, note

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _gpu_batches(g, w, keys_d, vals_d, a, e):
    lib, h = g._lib, g._h
    for i in range(a, e):
        rc = (lib.lsm_delete_batch(h, keys_d[i].data_ptr(), w.b) if w.is_delete[i]
              else lib.lsm_insert_batch(h, keys_d[i].data_ptr(), vals_d[i].data_ptr(), w.b))
        if rc:
            raise LSMError(rc, "update batch %d" % i)


def _oracle_batches(c, w, a, e):
    for i in range(a, e):
        if w.is_delete[i]:
            c.delete(w.keys[i])
        else:
            c.insert(w.keys[i], w.vals[i])


def _compare_level(g, c, i):
    gkv, gv = g.level(i)
    okv, ov = c.level(i)
    gkv, gv = host(gkv), host(gv)
    if not np.array_equal(gkv, okv):
        bad = np.flatnonzero(gkv != okv)
        raise AssertionError("level %d key variables differ at %d positions, first %d"
                             % (i, bad.size, bad[0]))
    assert np.array_equal(gv, ov), "level %d values differ" % i


def _queries(g, w, R, stage):
    """Every query of the workload on the GPU after the first R batches:
    properties on all of them, a sample against the filtered map oracle."""
    note("paper scale %s: queries" % stage)
    q_d = dev(w.lookups)
    lv, lf = g.lookup(q_d)
    cnt = g.count(dev(w.count_lo), dev(w.count_hi))
    rcnt = g.count(dev(w.range_lo), dev(w.range_hi))
    roff, rk, rv = g.range(dev(w.range_lo), dev(w.range_hi))
    torch.cuda.synchronize()
    lv, lf, cnt, rcnt = host(lv), host(lf), host(cnt), host(rcnt)
    roff, rk, rv = host(roff).astype(np.int64), host(rk), host(rv)

    check_range_properties(w.range_lo, w.range_hi, roff, rk, rcnt)
    samp = np.linspace(0, rk.size - 1, 50000).astype(np.int64)
    sv, sf = g.lookup(dev(rk[samp]))
    torch.cuda.synchronize()
    assert np.all(host(sf) == 1) and np.array_equal(host(sv), rv[samp]), "range pair != lookup"

    qi = np.linspace(0, w.lookups.size - 1, 20000).astype(np.int64)
    ci = np.linspace(0, w.count_lo.size - 1, 3000).astype(np.int64)
    ri = np.linspace(0, w.range_lo.size - 1, 3000).astype(np.int64)
    fm = FilteredMap(key_filter(w.lookups[qi], np.r_[w.count_lo[ci], w.range_lo[ri]],
                                np.r_[w.count_hi[ci], w.range_hi[ri]]))
    for i in range(R):
        if w.is_delete[i]:
            fm.delete(w.keys[i])
        else:
            fm.insert(w.keys[i], w.vals[i])
    ov, of = fm.m.lookup(w.lookups[qi])
    assert np.array_equal(lf[qi], of) and np.array_equal(lv[qi], ov), "sampled lookups differ"
    assert np.array_equal(cnt[ci], fm.m.count(w.count_lo[ci], w.count_hi[ci])), "sampled counts differ"
    oo, ok, oval = fm.m.range(w.range_lo[ri], w.range_hi[ri])
    gk, gvv, gsz = ranges_of(roff, rk, rv, ri)
    assert np.array_equal(np.diff(oo.astype(np.int64)), gsz), "sampled range sizes differ"
    assert np.array_equal(gk, ok) and np.array_equal(gvv, oval), "sampled range pairs differ"
    return lv, lf, cnt


def test_paper_scale_layout_and_sampled_queries():
    w = W.paper_scale()
    note("paper scale b=2^16: GPU build to r=1023")
    g = LSM(w.b)
    keys_d, vals_d = dev(w.keys), dev(w.vals)
    _gpu_batches(g, w, keys_d, vals_d, 0, 1023)
    g.sync()
    assert g.num_batches == 1023 and g.occupied() == list(range(10))

    note("paper scale: cascade oracle to r=1023")
    c = oracle.CascadeOracle(w.b)
    _oracle_batches(c, w, 0, 1023)
    for i in range(10):
        _compare_level(g, c, i)
    lv, lf, cnt = _queries(g, w, 1023, "r=1023 (levels 0-9)")
    assert 0.48 < lf.mean() < 0.52, lf.mean()

    note("paper scale: batch 1023 (the ten-level cascade)")
    _gpu_batches(g, w, keys_d, vals_d, 1023, 1024)
    _oracle_batches(c, w, 1023, 1024)
    g.sync()
    assert g.num_batches == 1024 and g.occupied() == [10]
    _compare_level(g, c, 10)
    n_valid = c.cleanup()
    cleaned = {i: c.level(i) for i in c.occupied()}
    r_clean = c.r
    del c

    lv, lf, cnt = _queries(g, w, 1024, "r=1024 (level 10)")
    assert 0.49 < lf.mean() < 0.51, lf.mean()
    assert 14.0 < cnt.mean() < 18.0, cnt.mean()

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
    lv2, lf2 = g.lookup(dev(w.lookups))
    torch.cuda.synchronize()
    assert np.array_equal(host(lf2), lf) and np.array_equal(host(lv2), lv)
    g.close()
