"""Parity of the batching form at the size the benchmark times: 4096 user
batches with log-normal sizes (median 4096, clipped to [256, 65536]),
uniform keys, every tenth a delete batch, at b = 2^16.

* Batched path (the benchmark's launch configuration: merges autotuned up to
  level 8): the user batches go through lsm_submit, packed in arrival order
  into about 426 LSM batches; every level is compared byte for byte with the
  cascade oracle fed the same packed batches (packing recomputed here).
* Plain path: one padded LSM batch per user batch (4096 batches, one level
  of 2^28 elements), compared byte for byte with the cascade oracle fed the
  same padded batches.
* Queries (2^20 lookups, 2^16 counts and 2^16 ranges of about 16 hits):
  both paths give identical answers on every query; properties hold on every
  range; a sample is compared with the map oracle fed the user batches'
  operations on the sampled keys, one after another.
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


def _answers(g, q_d, clo_d, chi_d, rlo_d, rhi_d):
    lv, lf = g.lookup(q_d)
    cnt = g.count(clo_d, chi_d)
    rcnt = g.count(rlo_d, rhi_d)
    roff, rk, rv = g.range(rlo_d, rhi_d)
    torch.cuda.synchronize()
    return [host(x) for x in (lv, lf, cnt, rcnt, roff, rk, rv)]


def test_batching_form_full_size():
    b = 1 << 16
    note("batching form full size: workload")
    ub = W.batching_stream(b=b)
    lk, clo, chi, rlo, rhi, width = W.batching_queries(ub)
    sizes = np.array([u[0].size for u in ub], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    allk = np.concatenate([u[0] for u in ub])
    allv = np.concatenate([u[1] for u in ub])
    dels = np.array([bool(u[2]) for u in ub])
    n_ops = int(offs[-1])
    kd, vd = dev(allk), dev(allv)

    note("batching form full size: batched path (%d ops)" % n_ops)
    gb = LSM(b)
    gb.autotune(max_level=8, reps=3)
    lib, h = gb._lib, gb._h
    for i in range(len(ub)):
        o = int(offs[i]) * 4
        rc = lib.lsm_submit(h, kd.data_ptr() + o, None if dels[i] else vd.data_ptr() + o,
                            int(sizes[i]), 1 if dels[i] else 0)
        if rc:
            raise LSMError(rc, "lsm_submit %d" % i)
    gb.flush()
    gb.sync()

    note("batching form full size: cascade oracle of the packed batches")
    status = np.repeat((~dels).astype(np.uint8), sizes)
    pv = np.where(status == 1, allv, 0).astype(np.uint32)
    c = oracle.CascadeOracle(b)
    for a in range(0, n_ops, b):
        c.insert_ordered(allk[a:a + b], pv[a:a + b], status[a:a + b])
    assert gb.num_batches == c.r == (n_ops + b - 1) // b
    assert gb.occupied() == c.occupied()
    for i in c.occupied():
        gkv, gv = gb.level(i)
        okv, ov = c.level(i)
        assert np.array_equal(host(gkv), okv), "batched level %d key variables differ" % i
        assert np.array_equal(host(gv), ov), "batched level %d values differ" % i
    del c

    note("batching form full size: plain path (4096 padded batches)")
    gp = LSM(b)
    lib, h = gp._lib, gp._h
    for i in range(len(ub)):
        o = int(offs[i]) * 4
        rc = (lib.lsm_delete_batch(h, kd.data_ptr() + o, int(sizes[i])) if dels[i]
              else lib.lsm_insert_batch(h, kd.data_ptr() + o, vd.data_ptr() + o, int(sizes[i])))
        if rc:
            raise LSMError(rc, "plain batch %d" % i)
    gp.sync()
    assert gp.num_batches == len(ub) and gp.occupied() == [12]
    note("batching form full size: cascade oracle of the padded batches")
    c = oracle.CascadeOracle(b)
    for k, v, dele in ub:
        if dele:
            c.delete(k)
        else:
            c.insert(k, v)
    gkv, gv = gp.level(12)
    okv, ov = c.level(12)
    assert np.array_equal(host(gkv), okv), "plain level 12 key variables differ"
    assert np.array_equal(host(gv), ov), "plain level 12 values differ"
    del c, gkv, gv, okv, ov

    note("batching form full size: queries")
    q_d, clo_d, chi_d, rlo_d, rhi_d = dev(lk), dev(clo), dev(chi), dev(rlo), dev(rhi)
    ab = _answers(gb, q_d, clo_d, chi_d, rlo_d, rhi_d)
    ap = _answers(gp, q_d, clo_d, chi_d, rlo_d, rhi_d)
    for x, y, name in zip(ab, ap, ("lookup values", "lookup flags", "counts", "range counts",
                                   "range offsets", "range keys", "range values")):
        assert np.array_equal(x, y), "batched and plain %s differ" % name
    lv, lf, cnt, rcnt, roff, rk, rv = ab
    roff = roff.astype(np.int64)
    check_range_properties(rlo, rhi, roff, rk, rcnt)
    assert 0.48 < lf.mean() < 0.52, lf.mean()
    assert 12.0 < cnt.mean() < 20.0, cnt.mean()

    qi = np.linspace(0, lk.size - 1, 20000).astype(np.int64)
    ci = np.linspace(0, clo.size - 1, 2000).astype(np.int64)
    ri = np.linspace(0, rlo.size - 1, 2000).astype(np.int64)
    fm = FilteredMap(key_filter(lk[qi], np.r_[clo[ci], rlo[ri]], np.r_[chi[ci], rhi[ri]]))
    for k, v, dele in ub:
        if dele:
            fm.delete(k)
        else:
            fm.insert(k, v)
    ov, of = fm.m.lookup(lk[qi])
    assert np.array_equal(lf[qi], of) and np.array_equal(lv[qi], ov), "sampled lookups differ"
    assert np.array_equal(cnt[ci], fm.m.count(clo[ci], chi[ci])), "sampled counts differ"
    oo, ok, oval = fm.m.range(rlo[ri], rhi[ri])
    gk, gvv, gsz = ranges_of(roff, rk, rv, ri)
    assert np.array_equal(np.diff(oo.astype(np.int64)), gsz), "sampled range sizes differ"
    assert np.array_equal(gk, ok) and np.array_equal(gvv, oval), "sampled range pairs differ"
    gb.close()
    gp.close()
