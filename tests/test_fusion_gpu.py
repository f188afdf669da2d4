"""GPU parity of the cascade fused into the top-digit sort: levels built with
fusion equal, byte for byte, both the cascade oracle's and those of the same
inserts with fusion off (pairwise merge launches).  Covers every fused depth
up to the default limit, partial batches and deletes, keys packed into one
top digit (one bucket holds the whole batch, so the fused merge ranks in
global memory), and a batch bucket larger than LDS (streaming sort, then the
global-memory merge).  Integer results, tolerance 0."""
import numpy as np
import pytest
import torch

from paper_1707_05354_amd.lsm import LSM
from _gpu import Trio, dev, host, note

pytestmark = pytest.mark.gpu


def run(b, batches, fusion, force_top=True, mode=LSM.SORT_TOP_DIGIT):
    t = Trio(b)
    if force_top:
        t.g.set_sort_path(mode)
    t.g.set_fusion(fusion)
    for kind, k, v in batches:
        if kind == "insert":
            t.insert(k, v)
        else:
            t.delete(k)
        t.check_levels()
    return t


def levels(t):
    t.g.sync()
    return {i: tuple(host(x).tobytes() for x in t.g.level(i)) for i in t.g.occupied()}


def stream(seed, b, R, domain, p_delete=0.25, partial=True):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(R):
        n = int(rng.integers(1, b + 1)) if partial and i % 3 == 1 else b
        k = rng.integers(0, domain, n, dtype=np.uint64).astype(np.uint32)
        if rng.random() < p_delete:
            out.append(("delete", k, None))
        else:
            out.append(("insert", k, rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)))
    return out


@pytest.mark.parametrize("b,R,domain", [(1, 300, 20), (3, 70, 1 << 31), (64, 40, 5000),
                                        (4096, 20, 1 << 31), (4099, 19, 1 << 14),
                                        (1 << 16, 17, 1 << 31)])
def test_fused_equals_pairwise_and_oracle(b, R, domain):
    note("fusion b=%d R=%d" % (b, R))
    ops = stream(1000 + b, b, R, domain)
    fused = run(b, ops, -1)
    plain = run(b, ops, 0)
    assert levels(fused) == levels(plain)
    rng = np.random.default_rng(b)
    q = rng.integers(0, domain, 600, dtype=np.uint64).astype(np.uint32)
    fused.check_queries(q, q[:200], (q[:200].astype(np.uint64) + domain // 40).astype(np.uint32))


@pytest.mark.parametrize("depth", [1, 2])
def test_partly_fused_cascades(depth):
    """Inserts deeper than the fusion limit: the sort fuses levels
    0..depth-1 into merge scratch and pairwise merges take it from there."""
    b, R = 64, 40
    note("partial fusion depth=%d" % depth)
    ops = stream(500 + depth, b, R, 3000)
    fused = run(b, ops, depth)
    plain = run(b, ops, 0)
    assert levels(fused) == levels(plain)


@pytest.mark.parametrize("b", [4096, 10000])
def test_fused_cascade_with_one_top_digit(b):
    """Keys below 2^20 share the top digit: one bucket holds every element,
    beyond what the fused merge ranks in LDS."""
    note("fusion one digit b=%d" % b)
    ops = stream(77 + b, b, 9, 1 << 20)
    fused = run(b, ops, -1)
    plain = run(b, ops, 0)
    assert levels(fused) == levels(plain)
