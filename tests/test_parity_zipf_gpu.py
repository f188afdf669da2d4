"""Parity on the Zipf batch-size sweep: keys Zipf(1.1) over [0, 2^24), 20%
delete batches, so hot keys are re-inserted and deleted many times and
within-batch duplicates are common (the last one must win).  Keys use the
24-bit sort (three digit passes)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import LSM
from _gpu import Trio, dev, host, note

pytestmark = pytest.mark.gpu

SWEEP_B = [1 << 13, 1 << 15, 1 << 17, 1 << 19]


@pytest.mark.parametrize("b", SWEEP_B)
def test_zipf_sweep_reduced(b):
    """n = 2^20 slots: every level and every query against the oracle."""
    w = W.zipf_sweep(b, n_total=1 << 20, nq=1 << 16)
    note("zipf reduced b=%d R=%d" % (b, w.R))
    t = Trio(b, key_bits=24)
    for i in range(w.R):
        if w.is_delete[i]:
            t.delete(w.keys[i])
        else:
            t.insert(w.keys[i], w.vals[i])
        if i % 8 == 7 or i == w.R - 1:
            t.check_levels()
    t.check_queries(w.lookups, w.count_lo[:4096], w.count_hi[:4096])
    t.check_queries(w.lookups[:16], w.range_lo[:4096], w.range_hi[:4096])


def _filtered_map(w, keep):
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


@pytest.mark.slow
@pytest.mark.parametrize("b", SWEEP_B)
def test_zipf_sweep_full_size(b):
    """n = 2^25 slots as the benchmark runs it: the occupied level byte for
    byte, sampled lookups against the map oracle replaying the sampled keys'
    own operations, and lookups of keys returned by range."""
    w = W.zipf_sweep(b)
    note("zipf full b=%d R=%d" % (b, w.R))
    g = LSM(b, key_bits=24)
    keys_d, vals_d = dev(w.keys), dev(w.vals)
    for i in range(w.R):
        if w.is_delete[i]:
            g.delete(keys_d[i])
        else:
            g.insert(keys_d[i], vals_d[i])
    g.sync()
    c = oracle.CascadeOracle(b)
    for i in range(w.R):
        if w.is_delete[i]:
            c.delete(w.keys[i])
        else:
            c.insert(w.keys[i], w.vals[i])
    assert g.occupied() == c.occupied()
    for lvl in c.occupied():
        okv, ov = c.level(lvl)
        gkv, gv = g.level(lvl)
        assert np.array_equal(host(gkv), okv), "level %d key variables" % lvl
        assert np.array_equal(host(gv), ov), "level %d values" % lvl
    del c
    lv, lf = g.lookup(dev(w.lookups))
    torch.cuda.synchronize()
    lv, lf = host(lv), host(lf)
    qi = np.linspace(0, w.lookups.size - 1, 20000).astype(np.int64)
    qs = np.unique(w.lookups[qi])
    m = _filtered_map(w, lambda k: np.isin(k, qs))
    ov, of = m.lookup(w.lookups[qi])
    assert np.array_equal(lf[qi], of) and np.array_equal(lv[qi], ov)
    off, rk, rv = g.range(dev(w.range_lo[:2000]), dev(w.range_hi[:2000]))
    sv, sf = g.lookup(rk)
    g.sync()
    assert np.all(host(sf) == 1) and np.array_equal(host(sv), host(rv))
    g.close()
