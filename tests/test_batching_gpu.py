"""GPU parity of the batching form: the coalescer packs user batches of any
size into LSM batches of b (arrival order, the newest operation on a key
wins), optionally inserting full batches by replaying captured hipGraphs,
with autotuned merge variants.  Every level is compared with the cascade
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


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("b,domain,max_len", [(7, 20, 25), (64, 300, 200), (4096, 20000, 9000)])
def test_coalescer_matches_oracle(b, domain, max_len, graphs):
    note("coalescer b=%d graphs=%s" % (b, graphs))
    g = LSM(b)
    g.use_graphs(graphs)
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


def test_graph_replays_equal_eager_inserts():
    """The same packed stream with graphs on and off gives identical levels
    after every batch (each graph is replayed many times, with eager work
    and synchronisation between replays)."""
    b = 2048
    note("graph vs eager b=2048")
    ga, gb = LSM(b), LSM(b)
    gb.use_graphs(True)
    stream = user_stream(77, b, 120, 50000, 3000)
    for t, (k, v, dele) in enumerate(stream):
        for gg in (ga, gb):
            gg.submit(dev(k), None if dele else dev(v), delete=dele)
        ga.sync()
        gb.sync()
        assert ga.num_batches == gb.num_batches
        for i in ga.occupied():
            ka, va = ga.level(i)
            kb, vb = gb.level(i)
            assert torch.equal(ka, kb) and torch.equal(va, vb), (t, i)
    ga.close()
    gb.close()


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
    g.use_graphs(True)
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
    gc.use_graphs(True)
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
