"""GPU parity of the batching form: the coalescer packs user batches of any
size into LSM batches of b (arrival order, the newest operation on a key
wins), with autotuned merge variants.  Every level is compared with the cascade
oracle fed the same packed batches (packing recomputed here, independently
of the library), and every query with the map oracle fed the user batches
one after another."""
import numpy as np
import pytest
import torch

import oracle
from paper_1707_05354_amd import workload as W
from paper_1707_05354_amd.lsm import LSM, LSMError, LSM_EKEY
from _gpu import dev, host, note

pytestmark = pytest.mark.gpu


class PackModel:
    """Oracle side of the coalescer: packs user batches into batches of b
    and feeds full ones (and flushed partial ones) to the cascade oracle."""

    def __init__(self, b):
        self.b = b
        self.c = oracle.CascadeOracle(b)
        self.m = oracle.MapOracle()
        self.k, self.v, self.s = [], [], []

    def submit(self, keys, vals, delete):
        if delete:
            self.m.delete(keys)
        else:
            self.m.insert(keys, vals)
        for j in range(len(keys)):
            self.k.append(int(keys[j]))
            self.v.append(0 if delete else int(vals[j]))
            self.s.append(0 if delete else 1)
            if len(self.k) == self.b:
                self.flush()

    def submit_mixed(self, keys, vals, is_del):
        """Arrival-ordered operations of both types.  The map oracle applies
        each run of consecutive operations of one type as one batch (a batch
        is applied element by element, in order, so this is the same as one
        operation at a time)."""
        cut = np.flatnonzero(np.diff(is_del.astype(np.int8))) + 1
        for a, e in zip(np.r_[0, cut], np.r_[cut, len(keys)]):
            if is_del[a]:
                self.m.delete(keys[a:e])
            else:
                self.m.insert(keys[a:e], vals[a:e])
        for j in range(len(keys)):
            self.k.append(int(keys[j]))
            self.v.append(0 if is_del[j] else int(vals[j]))
            self.s.append(0 if is_del[j] else 1)
            if len(self.k) == self.b:
                self.flush()

    def direct(self, kind, keys, vals=None, is_del=None):
        """A batch handed to lsm_insert/delete/update_batch: the staged
        elements are older, so they are inserted first as their own batch."""
        self.flush()
        if kind == "insert":
            self.m.insert(keys, vals)
            self.c.insert(keys, vals)
        elif kind == "delete":
            self.m.delete(keys)
            self.c.delete(keys)
        else:
            self.m.mixed(keys, vals, is_del)
            self.c.insert(keys, vals, (1 - np.asarray(is_del, np.uint8)).astype(np.uint8))

    def flush(self):
        if self.k:
            self.c.insert_ordered(np.array(self.k, np.uint32), np.array(self.v, np.uint32),
                                  np.array(self.s, np.uint8))
            self.k, self.v, self.s = [], [], []


def check_levels(g, model):
    g.sync()
    assert g.num_batches == model.c.r
    assert g.occupied() == model.c.occupied()
    for i in model.c.occupied():
        kv, v = g.level(i)
        okv, ov = model.c.level(i)
        assert np.array_equal(host(kv), okv), "level %d key variables" % i
        assert np.array_equal(host(v), ov), "level %d values" % i


def check_queries(g, model, q, lo, hi):
    model.flush()  # queries flush the staged elements first
    gv, gf = g.lookup(dev(q))
    gc = g.count(dev(lo), dev(hi))
    go, gk, gval = g.range(dev(lo), dev(hi))
    torch.cuda.synchronize()
    ov, of = model.m.lookup(q)
    assert np.array_equal(host(gf), of) and np.array_equal(host(gv), ov)
    assert np.array_equal(host(gc), model.m.count(lo, hi))
    oo, ok, oval = model.m.range(lo, hi)
    assert np.array_equal(host(go), oo)
    assert np.array_equal(host(gk), ok) and np.array_equal(host(gval), oval)


def user_stream(seed, b, nbatch, domain, max_len):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nbatch):
        n = int(rng.integers(1, max_len + 1))
        k = rng.integers(0, domain, n).astype(np.uint32)
        v = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        out.append((k, v, bool(rng.random() < 0.35)))
    return out


@pytest.mark.parametrize("b,domain,max_len", [(7, 20, 25), (64, 300, 200), (4096, 20000, 9000)])
def test_coalescer_matches_oracle(b, domain, max_len):
    note("coalescer b=%d" % b)
    g = LSM(b)
    model = PackModel(b)
    stream = user_stream(1000 + b, b, 60, domain, max_len)
    q = np.arange(domain + 2, dtype=np.uint32)
    lo = np.arange(0, domain, 3, dtype=np.uint32)
    hi = np.minimum(lo + 17, domain + 1).astype(np.uint32)
    for t, (k, v, dele) in enumerate(stream):
        g.submit(dev(k), None if dele else dev(v), delete=dele)
        model.submit(k, v, dele)
        assert g.pending == len(model.k)
        check_levels(g, model)
        if t % 20 == 19:
            check_queries(g, model, q, lo, hi)
            check_levels(g, model)
    g.flush()
    model.flush()
    check_levels(g, model)
    check_queries(g, model, q, lo, hi)
    g.close()


def test_staged_insert_then_direct_delete_of_the_same_key():
    """A key staged by lsm_submit and then deleted by lsm_delete_batch is
    gone: the staged insert is older, so it is inserted first."""
    b = 64
    note("staged insert, direct delete b=64")
    g = LSM(b)
    model = PackModel(b)
    k = np.array([5, 9, 13], np.uint32)
    v = np.array([50, 90, 130], np.uint32)
    g.submit(dev(k), dev(v))
    model.submit(k, v, False)
    assert g.pending == 3
    d = np.array([9], np.uint32)
    g.delete(dev(d))
    model.direct("delete", d)
    assert g.pending == 0 and g.num_batches == 2
    gv, gf = g.lookup(dev(np.array([5, 9, 13, 7], np.uint32)))
    torch.cuda.synchronize()
    assert host(gf).tolist() == [1, 0, 1, 0] and host(gv).tolist() == [50, 0, 130, 0]
    check_levels(g, model)
    check_queries(g, model, np.arange(20, dtype=np.uint32), np.array([0, 6], np.uint32),
                  np.array([10, 19], np.uint32))
    g.close()


@pytest.mark.parametrize("b", [5, 256, 4096])
def test_submit_paths_and_direct_batches_interleaved(b):
    """lsm_submit, lsm_submit_mixed and the three direct batch calls mixed
    on one handle, in random order and sizes: every level equals the
    cascade oracle fed the same batches (staged elements flushed before each
    direct batch) and the answers equal the map oracle."""
    note("interleaved submit / direct b=%d" % b)
    rng = np.random.default_rng(b)
    domain = 3 * b + 11
    g = LSM(b)
    model = PackModel(b)
    q = np.arange(domain + 2, dtype=np.uint32)
    lo = np.arange(0, domain, 5, dtype=np.uint32)
    hi = np.minimum(lo + 9, domain + 1).astype(np.uint32)
    for t in range(60):
        kind = rng.integers(0, 5)
        n = int(rng.integers(1, 2 * b + 1)) if kind < 2 else int(rng.integers(1, b + 1))
        k = rng.integers(0, domain, n).astype(np.uint32)
        v = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        dl = (rng.random(n) < 0.4).astype(np.uint8)
        if kind == 0:
            dele = bool(rng.random() < 0.3)
            g.submit(dev(k), None if dele else dev(v), delete=dele)
            model.submit(k, v, dele)
        elif kind == 1:
            g.submit_mixed(dev(k), dev(v), torch.from_numpy(dl).cuda())
            model.submit_mixed(k, v, dl)
        elif kind == 2:
            g.insert(dev(k), dev(v))
            model.direct("insert", k, v)
        elif kind == 3:
            g.delete(dev(k))
            model.direct("delete", k)
        else:
            g.update(dev(k), dev(v), torch.from_numpy(dl).cuda())
            model.direct("mixed", k, v, dl)
        assert g.pending == len(model.k), t
        if t % 10 == 9:
            check_levels(g, model)
            check_queries(g, model, q, lo, hi)
    g.flush()
    model.flush()
    check_levels(g, model)
    check_queries(g, model, q, lo, hi)
    g.close()


@pytest.mark.parametrize("variant", range(6))
def test_every_merge_variant_is_exact(variant):
    b = 1000
    note("merge variant %d" % variant)
    g = LSM(b)
    for lvl in range(12):
        g.set_tuning(lvl, variant)
    model = PackModel(b)
    for (k, v, dele) in user_stream(500 + variant, b, 40, 5000, 4000):
        g.submit(dev(k), None if dele else dev(v), delete=dele)
        model.submit(k, v, dele)
    g.flush()
    model.flush()
    check_levels(g, model)
    q = np.arange(5002, dtype=np.uint32)
    check_queries(g, model, q, q[:1000], q[:1000] + 40)
    g.close()


def test_autotune_then_exact():
    b = 4096
    note("autotune b=4096")
    g = LSM(b)
    g.autotune(max_level=6, reps=3)
    for lvl in range(7):
        v, us = g.tuning(lvl)
        assert 0 <= v < 6 and all(x > 0 for x in us)
        assert us[v] == min(us)
    model = PackModel(b)
    for (k, v, dele) in user_stream(9, b, 80, 100000, 9000):
        g.submit(dev(k), None if dele else dev(v), delete=dele)
        model.submit(k, v, dele)
    g.flush()
    model.flush()
    check_levels(g, model)
    g.close()


def test_checked_submit_rejects_bad_keys_without_staging():
    g = LSM(16, checked=True)
    k = np.arange(10, dtype=np.uint32)
    g.submit(dev(k), dev(k))
    bad = np.array([1, 2, 1 << 31], np.uint32)
    with pytest.raises(LSMError) as ei:
        g.submit(dev(bad), dev(bad))
    assert ei.value.status == LSM_EKEY
    assert g.pending == 10
    g.close()


def test_plain_and_batched_paths_answer_alike():
    """The same user batches through the plain path (one padded LSM batch
    per user batch) and through the coalescer give identical answers."""
    b = 1 << 12
    note("plain vs batched b=4096")
    ub = W.batching_stream(config=41, n_batches=300, median=1024, b=b)
    gp, gc = LSM(b), LSM(b)
    m = oracle.MapOracle()
    for k, v, dele in ub:
        kd = dev(k)
        if dele:
            for o in range(0, k.size, b):
                gp.delete(kd[o:o + b])
            gc.submit(kd, delete=True)
            m.delete(k)
        else:
            vd = dev(v)
            for o in range(0, k.size, b):
                gp.insert(kd[o:o + b], vd[o:o + b])
            gc.submit(kd, vd)
            m.insert(k, v)
    allk = np.concatenate([u[0] for u in ub])
    rng = np.random.default_rng(0)
    q = np.concatenate([allk[rng.integers(0, allk.size, 20000)],
                        rng.integers(0, 1 << 31, 20000).astype(np.uint32)])
    lo = rng.integers(0, (1 << 31) - 2000000, 3000).astype(np.uint32)
    hi = lo + 1000000
    ov, of = m.lookup(q)
    for g in (gp, gc):
        gv, gf = g.lookup(dev(q))
        torch.cuda.synchronize()
        assert np.array_equal(host(gf), of) and np.array_equal(host(gv), ov)
        assert np.array_equal(host(g.count(dev(lo), dev(hi))), m.count(lo, hi))
    gp.close()
    gc.close()
