"""Strong guarantee under allocation failure: with lsm_fail_alloc_after(n),
for every n up to the first that lets the call through, each update, range,
cleanup, bulk insert and coalesced submit that needs memory either returns
LSM_ENOMEM and leaves r and every occupied level byte for byte as they were,
or succeeds; once it succeeds the dictionary equals both oracles.  Integer
results, tolerance 0."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd.lsm import LSM_ENOMEM, LSMError
from _gpu import Trio, dev, host, note

pytestmark = pytest.mark.gpu


def snapshot(g):
    g.sync()
    return g.num_batches, {i: tuple(host(x).tobytes() for x in g.level(i)) for i in g.occupied()}


def run_until_success(t, gpu_call, oracle_call, max_n=40):
    """Calls gpu_call with 0, 1, 2, ... allocations allowed until it
    succeeds; every failure must be LSM_ENOMEM with the state unchanged."""
    before = snapshot(t.g)
    failures = 0
    for n in range(max_n):
        t.g.fail_alloc_after(n)
        try:
            gpu_call()
        except LSMError as e:
            assert e.status == LSM_ENOMEM, (n, e)
            assert snapshot(t.g) == before, "state changed by a failed call (n=%d)" % n
            failures += 1
            continue
        t.g.fail_alloc_after(-1)
        oracle_call()
        return failures
    raise AssertionError("the call never succeeded")


def stream(rng, b, n, domain):
    k = rng.integers(0, domain, n).astype(np.uint32)
    v = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return k, v


@pytest.mark.parametrize("op", ["insert", "delete", "mixed", "range", "cleanup", "bulk", "submit"])
def test_enomem_leaves_the_dictionary_unchanged(op):
    b = 1000
    note("enomem %s" % op)
    rng = np.random.default_rng(hash(op) % 1000)
    t = Trio(b)
    domain = 20000
    for _ in range(7):  # r = 7: levels 0-2 full, the next insert allocates level 3
        k, v = stream(rng, b, b, domain)
        t.insert(k, v)
    q = rng.integers(0, domain, 3000).astype(np.uint32)
    lo = rng.integers(0, domain, 400).astype(np.uint32)
    hi = (lo + 200).astype(np.uint32)
    k, v = stream(rng, b, b, domain)
    if op == "insert":
        fails = run_until_success(t, lambda: t.g.insert(dev(k), dev(v)),
                                  lambda: (t.m.insert(k, v), t.c.insert(k, v)))
    elif op == "delete":
        fails = run_until_success(t, lambda: t.g.delete(dev(k)),
                                  lambda: (t.m.delete(k), t.c.delete(k)))
    elif op == "mixed":
        dl = (rng.random(b) < 0.5).astype(np.uint8)
        fails = run_until_success(
            t, lambda: t.g.update(dev(k), dev(v), torch.from_numpy(dl).cuda()),
            lambda: (t.m.mixed(k, v, dl), t.c.insert(k, v, (1 - dl).astype(np.uint8))))
    elif op == "range":
        # More queries than any earlier call: the query scratch must grow.
        big_lo = rng.integers(0, domain, 100000).astype(np.uint32)
        big_hi = (big_lo + 50).astype(np.uint32)
        got = {}

        def call():
            got["r"] = t.g.range(dev(big_lo), dev(big_hi), cap=1 << 22)
        fails = run_until_success(t, call, lambda: None)
        torch.cuda.synchronize()
        oo, ok, ov = t.m.range(big_lo, big_hi)
        go, gk, gv = got["r"]
        assert np.array_equal(host(go), oo) and np.array_equal(host(gk), ok)
        assert np.array_equal(host(gv), ov)
    elif op == "cleanup":
        fails = run_until_success(t, lambda: t.g.cleanup(), lambda: t.c.cleanup())
    elif op == "bulk":
        kb, vb = stream(rng, b, 5 * b + 17, domain)

        def oracle_bulk():
            for a in range(0, kb.size, b):
                t.m.insert(kb[a:a + b], vb[a:a + b])
                t.c.insert(kb[a:a + b], vb[a:a + b])
        t.merge_count_comparable = False
        fails = run_until_success(t, lambda: t.g.bulk_insert(dev(kb), dev(vb)), oracle_bulk)
    else:  # submit: fills one staged batch (inserted at once) and stages the rest
        ks, vs = stream(rng, b, b + 300, domain)

        def oracle_submit():
            t.m.insert(ks, vs)
            t.c.insert_ordered(ks[:b], vs[:b], np.ones(b, np.uint8))
        fails = run_until_success(t, lambda: t.g.submit(dev(ks), dev(vs)), oracle_submit)
        assert t.g.pending == 300
        t.g.flush()
        t.c.insert_ordered(ks[b:], vs[b:], np.ones(300, np.uint8))
    assert fails >= 1, "the call allocated nothing, so no failure was injected"
    t.check_levels()
    t.check_queries(q, lo, hi)
    t.g.close()
