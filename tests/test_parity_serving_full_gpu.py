"""Parity of the serving form at the size the benchmark serves: a resident
dictionary of 2^28 pairs (4096 insert batches of b = 2^16, level 12), then
the benchmark's 40000 requests (50% lookup, 10% count, 10% range, 25%
insert, 5% delete; sizes log-uniform in [1, 8192]) served at saturation by
the continuous-batching loop.

* The resident level 12 (2^28 elements, 2 GiB) is compared byte for byte
  with the cascade oracle.
* A sample of query requests of every kind, spread over the run, is
  compared with the epoch-log oracle: the map oracle fed, in order, the
  resident batches and then each epoch's update requests in arrival order,
  restricted to the keys the sample can see (exact for those requests, see
  _fullsize); each sampled request is answered against the state after the
  epochs before its own.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import LSM, LSMError
from paper_1707_05354_amd.serving import COUNT, DELETE, INSERT, LOOKUP, RANGE, Server
from _fullsize import ops_touching
from _gpu import dev, host, note

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _same(x, y):
    if isinstance(x, tuple):
        return all(np.array_equal(np.asarray(p).astype(np.int64), np.asarray(q).astype(np.int64))
                   for p, q in zip(x, y))
    return np.array_equal(np.asarray(x).astype(np.int64), np.asarray(y).astype(np.int64))


def test_serving_form_full_size():
    b, R = 1 << 16, 4096
    note("serving full size: workload")
    rk, rv = W.resident(b=b, R=R)
    reqs = W.serving_requests(rk, 40000, rate=1.0)

    note("serving full size: resident build (2^28 pairs)")
    g = LSM(b)
    kd, vd = dev(rk), dev(rv)
    lib, h = g._lib, g._h
    for i in range(R):
        rc = lib.lsm_insert_batch(h, kd[i].data_ptr(), vd[i].data_ptr(), b)
        if rc:
            raise LSMError(rc, "resident batch %d" % i)
    g.sync()
    assert g.num_batches == R and g.occupied() == [12]
    del kd, vd
    torch.cuda.empty_cache()

    note("serving full size: cascade oracle of the resident build")
    c = oracle.CascadeOracle(b)
    for i in range(R):
        c.insert(rk[i], rv[i])
    gkv, gv = g.level(12)
    okv, ov = c.level(12)
    assert np.array_equal(host(gkv), okv), "resident level 12 key variables differ"
    assert np.array_equal(host(gv), ov), "resident level 12 values differ"
    del c, gkv, gv, okv, ov

    # A sample of every query kind, spread over the arrival order.
    sample = []
    for kind in (LOOKUP, COUNT, RANGE):
        idx = np.flatnonzero(reqs.kind == kind)
        sample.extend(idx[np.linspace(0, idx.size - 1, 80).astype(np.int64)].tolist())
    sample = np.unique(np.array(sample, np.int64))
    is_sampled = np.zeros(reqs.n, bool)
    is_sampled[sample] = True

    note("serving full size: serve %d requests at saturation" % reqs.n)
    srv = Server(g, reqs, max_epoch_ops=1 << 20, in_flight=3,
                 capture_ranges=lambda a, e: bool(is_sampled[a:e].any()))
    res = srv.run(realtime=False)
    assert len(res.epochs) >= 10
    assert sum(ep.last - ep.first for ep in res.epochs) == reqs.n

    note("serving full size: epoch-log oracle of %d sampled requests" % sample.size)
    pts, lo, hi = [], [], []
    for q in sample:
        a, n = int(reqs.off[q]), int(reqs.size[q])
        if reqs.kind[q] == LOOKUP:
            pts.append(reqs.lookup_keys[a:a + n])
        elif reqs.kind[q] == COUNT:
            lo.append(reqs.count_lo[a:a + n])
            hi.append(reqs.count_hi[a:a + n])
        else:
            lo.append(reqs.range_lo[a:a + n])
            hi.append(reqs.range_hi[a:a + n])
    pts, lo, hi = np.concatenate(pts), np.concatenate(lo), np.concatenate(hi)
    m = oracle.MapOracle()
    sel = ops_touching(rk, pts, lo, hi)  # resident operations, in batch order
    m.insert(rk.reshape(-1)[sel], rv.reshape(-1)[sel])
    usel = ops_touching(reqs.upd_keys, pts, lo, hi)  # update operations, in arrival order
    checked = 0
    for ep in res.epochs:
        for q in range(ep.first, ep.last):
            if not is_sampled[q]:
                continue
            k, a, n = int(reqs.kind[q]), int(reqs.off[q]), int(reqs.size[q])
            if k == LOOKUP:
                exp = m.lookup(reqs.lookup_keys[a:a + n])
            elif k == COUNT:
                exp = m.count(reqs.count_lo[a:a + n], reqs.count_hi[a:a + n])
            else:
                off, keys, vals = m.range(reqs.range_lo[a:a + n], reqs.range_hi[a:a + n])
                exp = (off.astype(np.int64), keys, vals)
            assert _same(srv.results(res, q), exp), (q, k)
            checked += 1
        upd = np.flatnonzero((reqs.kind[ep.first:ep.last] == INSERT) |
                             (reqs.kind[ep.first:ep.last] == DELETE)) + ep.first
        if upd.size:
            # The epoch's update operations, [a, e) of the update stream,
            # restricted to the sampled keys and applied in arrival order
            # (runs of one type as one batch, element by element).
            a = int(reqs.off[upd[0]])
            e = int(reqs.off[upd[-1]] + reqs.size[upd[-1]])
            ops = usel[(usel >= a) & (usel < e)]
            dl = reqs.upd_is_del[ops].astype(bool)
            cut = np.flatnonzero(np.diff(dl.astype(np.int8))) + 1
            for x, y in zip(np.r_[0, cut], np.r_[cut, ops.size]):
                if x == y:
                    continue
                if dl[x]:
                    m.delete(reqs.upd_keys[ops[x:y]])
                else:
                    m.insert(reqs.upd_keys[ops[x:y]], reqs.upd_val[ops[x:y]])
    assert checked == sample.size
    g.close()
