#!/usr/bin/env python
"""Benchmark of the batched LSM dictionary on one MI355X.

One step = the whole hot path over one synthetic workload, from an empty
dictionary: 1024 update batches of b = 2^16 (n = 2^26 slots; batch i deletes
iff i mod 10 == 9), then 2^22 lookups, 2^20 count and 2^20 range queries
(about 16 hits each).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `value` is M updates/s over the update phase of the
timed steps; lookups, counts and ranges are reported beside it.  Every
kernel is timed per launch with HIP start/stop events on the dictionary's
stream; the roofline object covers the kernel with the largest share of
device time.  The CPU baseline is the oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "M updates/s and M lookups/s at b=2^16, n=2^26; % of HBM peak; p99 latency"


def log(msg: str) -> None:
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s: float = 15.0):
    """The oracle as it stands (std::map, one operation at a time) on the
    first batches of the same workload, stopping once ~budget_s is spent."""
    import oracle

    m = oracle.MapOracle()
    t0 = time.perf_counter()
    nb = 0
    while nb < w.R and time.perf_counter() - t0 < budget_s:
        if w.is_delete[nb]:
            m.delete(w.keys[nb])
        else:
            m.insert(w.keys[nb], w.vals[nb])
        nb += 1
    t_upd = time.perf_counter() - t0
    nq = min(w.lookups.size, 1 << 20)
    t1 = time.perf_counter()
    m.lookup(w.lookups[:nq])
    t_lk = time.perf_counter() - t1
    return {
        "value": round(nb * w.b / t_upd / 1e6, 3),
        "unit": "M updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d of %d update batches (%d ops, std::map one op at a time), then %d "
                  "lookups on that map: %.2f M lookups/s" % (nb, w.R, nb * w.b, nq, nq / t_lk / 1e6),
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
        "seconds": round(t_upd + t_lk, 2),
    }


def zipf_sweep(torch, L, W, reps: int = 2):
    """Batch-size sweep at n = 2^25 slots: b in {2^13, 2^15, 2^17, 2^19}, Zipf(1.1)
    keys over [0, 2^24) (24-bit sort), 20% delete batches, then 2^22 Zipf
    lookups.  Best of `reps` builds per point."""
    res = []
    for lb in (13, 15, 17, 19):
        b = 1 << lb
        t0 = time.perf_counter()
        w = W.zipf_sweep(b)
        log("sweep b=2^%d: workload ready in %.1f s" % (lb, time.perf_counter() - t0))
        kd = torch.from_numpy(w.keys.view(np.int32)).cuda()
        vd = torch.from_numpy(w.vals.view(np.int32)).cuda()
        qd = torch.from_numpy(w.lookups.view(np.int32)).cuda()
        lv = torch.empty(qd.numel(), dtype=torch.int32, device="cuda")
        lf = torch.empty(qd.numel(), dtype=torch.uint8, device="cuda")
        g = L.LSM(b, key_bits=24)
        lib, h = g._lib, g._h
        rows_k = [kd[i].data_ptr() for i in range(w.R)]
        rows_v = [vd[i].data_ptr() for i in range(w.R)]
        best_u, best_l = None, None
        for _ in range(reps):
            g.clear()
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            for i in range(w.R):
                rc = (lib.lsm_delete_batch(h, rows_k[i], b) if w.is_delete[i]
                      else lib.lsm_insert_batch(h, rows_k[i], rows_v[i], b))
                if rc:
                    raise L.LSMError(rc, "sweep update")
            rc = lib.lsm_flush(h)  # the last pending insertion belongs to the update phase
            if rc:
                raise L.LSMError(rc, "sweep flush")
            e[1].record()
            g.lookup(qd, out=(lv, lf))
            e[2].record()
            torch.cuda.synchronize()
            u, l = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
            best_u = u if best_u is None else min(best_u, u)
            best_l = l if best_l is None else min(best_l, l)
        g.sync()
        res.append({"b": b, "batches": w.R, "levels": g.occupied(),
                    "M_updates_per_s": round(w.R * b / (best_u * 1e-3) / 1e6, 2),
                    "M_lookups_per_s": round(qd.numel() / (best_l * 1e-3) / 1e6, 2),
                    "lookup_hit_rate": round(float(lf.float().mean().item()), 4)})
        log("sweep b=2^%d: %s" % (lb, res[-1]))
        g.close()
    return res


def cleanup_form(torch, L, W, reps: int = 2):
    """Cleanup (sec. III-E / IV-D) at the sizes of sec. V-E: n = 63 b with
    b = 2^20 and n = 127 b with b = 2^19, 10 % and 50 % of the resident
    elements stale (replaced duplicates); elements processed per second =
    resident elements / cleanup time (whole call, host read-back included).
    Then the query effect at b = 2^18, n = 127 b, 10 % stale: 2^25 lookups
    before, cleanup, the same lookups after."""
    res = {"points": []}
    for lb, R, stale in ((20, 63, 0.1), (20, 63, 0.5), (19, 127, 0.1), (19, 127, 0.5)):
        b = 1 << lb
        w = W.cleanup_build(b, R, stale, nq=1 << 10)
        kd = torch.from_numpy(w.keys.view(np.int32)).cuda()
        vd = torch.from_numpy(w.vals.view(np.int32)).cuda()
        g = L.LSM(b)
        best, v = None, 0
        for rep in range(reps + 1):
            g.clear()
            for i in range(R):
                g.insert(kd[i], vd[i])
            g.sync()
            torch.cuda.synchronize()
            if rep == reps:
                g.profile(True)
                g.profile_read(reset=True)
            t0 = time.perf_counter()
            v = g.cleanup()
            dt = time.perf_counter() - t0
            if rep < reps:
                best = dt if best is None else min(best, dt)
        prof = g.profile_read(reset=True)
        g.profile(False)
        ks = {}
        for k, name in enumerate(L.KERNEL_NAMES):
            if prof.launches[k]:
                ks[name] = {"launches": int(prof.launches[k]), "ms": round(prof.kernel_ms[k], 3),
                            "GB_per_s": round(prof.kernel_bytes[k] / max(1e-12, prof.kernel_ms[k] * 1e-3) / 1e9, 1)}
        byts = sum(prof.kernel_bytes)
        kms = sum(prof.kernel_ms)
        res["points"].append({
            "b": b, "batches": R, "resident": R * b, "valid": v,
            "removed_frac": round(1 - v / (R * b), 4), "levels_after": g.occupied(),
            "ms": round(best * 1e3, 3), "M_elements_per_s": round(R * b / best / 1e6, 1),
            "kernel_ms": round(kms, 3), "algorithmic_GB_per_s": round(byts / max(1e-12, kms * 1e-3) / 1e9, 1),
            "kernels": ks})
        log("cleanup: %s" % res["points"][-1])
        g.close()
        del kd, vd
    b, R = 1 << 18, 127
    w = W.cleanup_build(b, R, 0.1, nq=1 << 25)
    kd = torch.from_numpy(w.keys.view(np.int32)).cuda()
    vd = torch.from_numpy(w.vals.view(np.int32)).cuda()
    qd = torch.from_numpy(w.lookups.view(np.int32)).cuda()
    lv = torch.empty(qd.numel(), dtype=torch.int32, device="cuda")
    lf = torch.empty(qd.numel(), dtype=torch.uint8, device="cuda")
    g = L.LSM(b)
    for i in range(R):
        g.insert(kd[i], vd[i])
    g.lookup(qd, out=(lv, lf))
    g.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.lookup(qd, out=(lv, lf))
    torch.cuda.synchronize()
    before = time.perf_counter() - t0
    f_before = lf.clone()
    levels_before = g.occupied()
    t0 = time.perf_counter()
    g.cleanup()
    clean = time.perf_counter() - t0
    t0 = time.perf_counter()
    g.lookup(qd, out=(lv, lf))
    torch.cuda.synchronize()
    after = time.perf_counter() - t0
    assert bool(torch.equal(f_before, lf))
    res["lookups"] = {"b": b, "batches": R, "lookups": qd.numel(), "levels_before": levels_before,
                      "levels_after": g.occupied(), "before_ms": round(before * 1e3, 3),
                      "cleanup_ms": round(clean * 1e3, 3), "after_ms": round(after * 1e3, 3),
                      "speedup_incl_cleanup": round(before / (clean + after), 2),
                      "hit_rate": round(float(lf.float().mean().item()), 4)}
    log("cleanup lookups: %s" % res["lookups"])
    g.close()
    res["context"] = ("paper (K40c): cleanup 1870.2 / 1828.2 M elements/s at n=63*2^20 with "
                      "10 / 50 % removed; 1842.5 / 1794.3 at n=127*2^19; at b=2^18, n=127b, "
                      "32 M lookups 4.8x faster after cleanup, cleanup time included")
    return res


def bulk_form(torch, L, W, reps: int = 2):
    """Bulk build (sec. V-B): n uniform pairs loaded into an empty dictionary
    with one lsm_bulk_insert call (b = 2^16; n = 2^26 and the 2^28 resident
    set of the serving form), against the same pairs as 1024 / 4096
    sequential insert batches.  Elements per second, whole call."""
    res = []
    for R in (1024, 4096):
        b = 1 << 16
        n = R * b
        kd = torch.from_numpy(W.uniform_keys(7, 1, 0, n).view(np.int32)).cuda()
        vd = torch.from_numpy(W.values(7, 2, 0, n).view(np.int32)).cuda()
        g = L.LSM(b)
        lib, h = g._lib, g._h
        best_bulk, best_seq = None, None
        for _ in range(reps):
            g.clear()
            g.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.bulk_insert(kd, vd)
            dt = time.perf_counter() - t0
            best_bulk = dt if best_bulk is None else min(best_bulk, dt)
            levels = g.occupied()
            g.clear()
            g.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(R):
                rc = lib.lsm_insert_batch(h, kd.data_ptr() + 4 * i * b, vd.data_ptr() + 4 * i * b, b)
                if rc:
                    raise L.LSMError(rc, "insert")
            g.sync()
            dt = time.perf_counter() - t0
            best_seq = dt if best_seq is None else min(best_seq, dt)
        res.append({"b": b, "pairs": n, "levels": levels,
                    "bulk_ms": round(best_bulk * 1e3, 3),
                    "bulk_M_elements_per_s": round(n / best_bulk / 1e6, 1),
                    "sequential_ms": round(best_seq * 1e3, 3),
                    "sequential_M_elements_per_s": round(n / best_seq / 1e6, 1)})
        log("bulk: %s" % res[-1])
        g.close()
        del kd, vd
    return {"points": res, "context": "paper (K40c): bulk build 770 M elements/s (key-value radix sort)"}


def batching_form(torch, L, W, reps: int = 2):
    """4096 user batches, log-normal sizes (median 4096, sigma 1, clipped to
    [256, 65536]), uniform keys, every tenth a delete batch: the plain path
    (one padded LSM batch of b = 2^16 per user batch) against the batching
    form (coalescer packing into ~426 LSM batches, autotuned merges).  Best
    of `reps` runs of each; user ops per second."""
    b = 1 << 16
    t0 = time.perf_counter()
    ub = W.batching_stream(b=b)
    sizes = [u[0].size for u in ub]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    allk = np.concatenate([u[0] for u in ub])
    allv = np.concatenate([u[1] for u in ub])
    kd = torch.from_numpy(allk.view(np.int32)).cuda()
    vd = torch.from_numpy(allv.view(np.int32)).cuda()
    kp, vp = kd.data_ptr(), vd.data_ptr()
    dels = [u[2] for u in ub]
    n_ops = int(offs[-1])
    log("batching: %d user batches, %d ops, ready in %.1f s" % (len(ub), n_ops, time.perf_counter() - t0))

    def run(g, batched):
        lib, h = g._lib, g._h
        best = None
        for _ in range(reps):
            g.clear()
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            for i, n in enumerate(sizes):
                o = int(offs[i]) * 4
                if batched:
                    rc = lib.lsm_submit(h, kp + o, None if dels[i] else vp + o, n, 1 if dels[i] else 0)
                elif dels[i]:
                    rc = lib.lsm_delete_batch(h, kp + o, n)
                else:
                    rc = lib.lsm_insert_batch(h, kp + o, vp + o, n)
                if rc:
                    raise L.LSMError(rc, "batching run")
            if batched:
                g.flush()
            e[1].record()
            torch.cuda.synchronize()
            ms = e[0].elapsed_time(e[1])
            best = ms if best is None else min(best, ms)
        g.sync()
        return best, g.num_batches

    gp = L.LSM(b)
    plain_ms, plain_r = run(gp, False)
    gp.close()
    gb = L.LSM(b)
    t0 = time.perf_counter()
    gb.autotune(max_level=8, reps=3)
    tune_s = time.perf_counter() - t0
    tuning = [gb.tuning(i)[0] for i in range(9)]
    batch_ms, batch_r = run(gb, True)
    gb.close()
    res = {
        "user_batches": len(ub), "user_ops": n_ops,
        "plain": {"lsm_batches": plain_r, "ms": round(plain_ms, 3),
                  "M_user_ops_per_s": round(n_ops / (plain_ms * 1e-3) / 1e6, 2)},
        "batched": {"lsm_batches": batch_r, "ms": round(batch_ms, 3),
                    "M_user_ops_per_s": round(n_ops / (batch_ms * 1e-3) / 1e6, 2),
                    "merge_variant_by_level": tuning,
                    "autotune_s": round(tune_s, 2)},
        "speedup": round(plain_ms / batch_ms, 2),
    }
    log("batching: %s" % res)
    return res


def serving_form(torch, L, W, n_requests: int = 40000, loads=(0.25, 0.5, 0.75, 0.9)):
    """Resident dictionary of 2^28 pairs (4096 insert batches of 2^16),
    Poisson arrivals of mixed requests (50% lookup, 10% count, 10% range of
    width 256 (~32 hits), 25% insert, 5% delete; sizes log-uniform in
    [1, 8192]), served by the continuous-batching loop.  First a saturation
    run (everything arrived at t = 0) gives the capacity; the offered loads
    are then the given fractions of it.
    Reports throughput and p50/p99 request latency (completion - arrival)
    per point."""
    from paper_1707_05354_amd import serving as S

    b, R = 1 << 16, 4096
    t0 = time.perf_counter()
    rk, rv = W.resident(b=b, R=R)
    reqs = W.serving_requests(rk, n_requests, rate=1.0)
    base_t = reqs.t_arrive.copy()
    kd = torch.from_numpy(rk.view(np.int32)).cuda()
    vd = torch.from_numpy(rv.view(np.int32)).cuda()
    log("serving: resident %d pairs, %d requests (%d ops) ready in %.1f s"
        % (R * b, n_requests, int(reqs.size.sum()), time.perf_counter() - t0))
    g = L.LSM(b)
    lib, h = g._lib, g._h
    rows_k = [kd[i].data_ptr() for i in range(R)]
    rows_v = [vd[i].data_ptr() for i in range(R)]

    def rebuild():
        g.clear()
        for i in range(R):
            rc = lib.lsm_insert_batch(h, rows_k[i], rows_v[i], b)
            if rc:
                raise L.LSMError(rc, "resident build")
        g.sync()

    def serve(realtime):
        rebuild()
        srv = S.Server(g, reqs, max_epoch_ops=1 << 20, in_flight=3)
        res = srv.run(realtime=realtime)
        span = max(res.completion_s.max() - (reqs.t_arrive[0] if realtime else 0.0), 1e-9)
        del srv
        return res, span

    t1 = time.perf_counter()
    reqs.t_arrive = np.zeros_like(base_t)
    res, span = serve(False)
    cap_rps = n_requests / span
    sat = {"offered_rps": None, "throughput_rps": round(cap_rps), "M_ops_per_s": round(res.ops / span / 1e6, 2),
           **{k: round(v, 3) for k, v in S.percentiles(res.latency_s).items()}, "epochs": len(res.epochs)}
    log("serving saturation: %s" % sat)
    points = [dict(sat, load="saturation")]
    for f in loads:
        rate = f * cap_rps
        reqs.t_arrive = base_t / rate
        res, span = serve(True)
        p = {"load": f, "offered_rps": round(rate), "throughput_rps": round(n_requests / span),
             "M_ops_per_s": round(res.ops / span / 1e6, 2),
             **{k: round(v, 3) for k, v in S.percentiles(res.latency_s).items()},
             "epochs": len(res.epochs)}
        log("serving load %.2f: %s" % (f, p))
        points.append(p)
    g.close()
    return {"resident_pairs": R * b, "requests": n_requests, "ops": int(reqs.size.sum()),
            "mix": "50%% lookup, 10%% count, 10%% range (width %d), 25%% insert, 5%% delete" % reqs.width,
            "points": points, "seconds": round(time.perf_counter() - t1, 1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batches", type=int, default=1024, help="update batches per step")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the Zipf batch-size sweep (b = 2^13..2^19 at n = 2^25)")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batching-form comparison (4096 log-normal user batches)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving form (resident 2^28 pairs, offered-load sweep)")
    ap.add_argument("--no-cleanup", action="store_true",
                    help="skip the cleanup measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 4 times (PMC byte calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    from paper_1707_05354_amd import lsm as L
    from paper_1707_05354_amd import workload as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": 1 << 28,
                          "bytes_written_per_copy": 1 << 28, "copies": 4}))
        return 0
    t0 = time.perf_counter()
    w = W.paper_scale(R=args.batches)
    log("workload generated in %.1f s: %s" % (time.perf_counter() - t0, w.name))

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()

    keys_d, vals_d = dev(w.keys), dev(w.vals)
    q_d = dev(w.lookups)
    clo_d, chi_d = dev(w.count_lo), dev(w.count_hi)
    rlo_d, rhi_d = dev(w.range_lo), dev(w.range_hi)
    nq, nc, nr = q_d.numel(), clo_d.numel(), rlo_d.numel()
    lv = torch.empty(nq, dtype=torch.int32, device="cuda")
    lf = torch.empty(nq, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(nc, dtype=torch.int32, device="cuda")
    roff = torch.empty(nr + 1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    g = L.LSM(w.b)
    lib, h = g._lib, g._h
    b = w.b
    row_k = [keys_d[i].data_ptr() for i in range(w.R)]
    row_v = [vals_d[i].data_ptr() for i in range(w.R)]
    is_del = [bool(x) for x in w.is_delete]
    cap = [1 << 20]
    rk = [torch.empty(cap[0], dtype=torch.int32, device="cuda")]
    rv = [torch.empty(cap[0], dtype=torch.int32, device="cuda")]
    total = ctypes.c_uint64(0)

    def updates(R=w.R):
        for i in range(R):
            rc = (lib.lsm_delete_batch(h, row_k[i], b) if is_del[i]
                  else lib.lsm_insert_batch(h, row_k[i], row_v[i], b))
            if rc:
                raise L.LSMError(rc, "update batch %d" % i)
        # The last batch's second half (bucket sort and cascade) belongs to
        # the update phase: enqueue it before the phase's end event.
        rc = lib.lsm_flush(h)
        if rc:
            raise L.LSMError(rc, "lsm_flush")

    def ranges():
        rc = lib.lsm_range(h, rlo_d.data_ptr(), rhi_d.data_ptr(), nr, roff.data_ptr(),
                           rk[0].data_ptr(), rv[0].data_ptr(), cap[0], ctypes.byref(total))
        if rc == L.LSM_ECAPACITY:
            cap[0] = int(total.value) + (1 << 20)
            rk[0] = torch.empty(cap[0], dtype=torch.int32, device="cuda")
            rv[0] = torch.empty(cap[0], dtype=torch.int32, device="cuda")
            rc = lib.lsm_range(h, rlo_d.data_ptr(), rhi_d.data_ptr(), nr, roff.data_ptr(),
                               rk[0].data_ptr(), rv[0].data_ptr(), cap[0], ctypes.byref(total))
        if rc:
            raise L.LSMError(rc, "lsm_range")

    def step(ev):
        g.clear()
        ev[0].record()
        updates()
        ev[1].record()
        g.lookup(q_d, out=(lv, lf))
        ev[2].record()
        g.count(clo_d, chi_d, out=cnt)
        ev[3].record()
        ranges()
        ev[4].record()

    for i in range(args.warmup):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        step(ev)
        torch.cuda.synchronize()
        log("warmup step %d: %.1f ms" % (i, ev[0].elapsed_time(ev[4])))

    # Timed steps: no per-kernel instrumentation, phases bracketed by events.
    phase = np.zeros(4)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        step(ev)
        torch.cuda.synchronize()
        ph = [ev[k].elapsed_time(ev[k + 1]) for k in range(4)]
        phase += ph
        log("step %d: updates %.2f ms, lookups %.2f ms, counts %.2f ms, ranges %.2f ms"
            % (i, *ph))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    # One more step of the same workload with every kernel launch bracketed by
    # HIP start/stop events (hipExtLaunchKernelGGL) for the per-kernel table.
    g.profile(True)
    g.profile_read(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    step(ev)
    prof = g.profile_read(reset=True)
    g.profile(False)
    g.sync()
    log("profiled step: %.1f ms" % ev[0].elapsed_time(ev[4]))

    # The same queries with levels 0-9 all full (r = 1023: the multi-level
    # case of the paper's query tables; the step itself queries one level,
    # the best case).  Best of two runs each, outside the timed steps.
    g.clear()
    updates(w.R - 1)
    g.sync()
    torch.cuda.synchronize()
    levels_1023 = g.occupied()

    def best_ms(fn, reps=2):
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return best

    lk1 = best_ms(lambda: g.lookup(q_d, out=(lv, lf)))
    hits1 = float(lf.float().mean().item())
    ct1 = best_ms(lambda: g.count(clo_d, chi_d, out=cnt))
    mean1 = float(cnt.float().mean().item())
    rg1 = best_ms(ranges)
    r1023 = {"batches": w.R - 1, "levels": levels_1023,
             "lookups": {"value": round(nq / (lk1 * 1e-3) / 1e6, 2), "unit": "M lookups/s",
                         "hit_rate": round(hits1, 4)},
             "counts": {"value": round(nc / (ct1 * 1e-3) / 1e6, 2), "unit": "M counts/s",
                        "mean_count": round(mean1, 3)},
             "ranges": {"value": round(nr / (rg1 * 1e-3) / 1e6, 2), "unit": "M ranges/s",
                        "pairs_returned": int(total.value)}}
    log("queries at r=1023: %s" % r1023)
    g.clear()
    updates()
    g.sync()

    # Order queries (successor / predecessor) on the final state, same keys
    # as the lookups; best of two runs each, outside the step.
    ok_ = torch.empty(nq, dtype=torch.int32, device="cuda")
    ov_ = torch.empty(nq, dtype=torch.int32, device="cuda")
    of_ = torch.empty(nq, dtype=torch.uint8, device="cuda")
    order = {}
    for name in ("successor", "predecessor"):
        fn = getattr(lib, "lsm_" + name)
        best = None
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rc = fn(h, q_d.data_ptr(), nq, ok_.data_ptr(), ov_.data_ptr(), of_.data_ptr())
            e1.record()
            torch.cuda.synchronize()
            if rc:
                raise L.LSMError(rc, name)
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        order[name] = {"value": round(nq / (best * 1e-3) / 1e6, 2), "unit": "M queries/s",
                       "found_rate": round(float(of_.float().mean().item()), 4)}
    log("order queries: %s" % order)

    K = args.steps
    upd_ms, lk_ms, ct_ms, rg_ms = (phase / K).tolist()
    n_upd = w.R * w.b
    hits = float(lf.float().mean().item())
    mean_count = float(cnt.float().mean().item())
    range_total = int(total.value)

    kernels = {}
    for k, name in enumerate(L.KERNEL_NAMES):
        n = int(prof.launches[k])
        if n == 0:
            continue
        ms = prof.kernel_ms[k]
        kernels[name] = {
            "launches_per_step": n,
            "avg_us": round(ms / n * 1e3, 3),
            "ms_per_step": round(ms, 3),
            "GB_per_s": round(prof.kernel_bytes[k] / (ms * 1e-3) / 1e9, 1) if prof.kernel_bytes[k] else None,
        }
    # Roofline of the kernel with the largest share of device time.
    dom = max(range(len(L.KERNEL_NAMES)), key=lambda k: prof.kernel_ms[k])
    dom_bytes, dom_ms, dom_n = prof.kernel_bytes[dom], prof.kernel_ms[dom], int(prof.launches[dom])
    dom_gbs = dom_bytes / (dom_ms * 1e-3) / 1e9
    # HBM bytes per launch from the committed counter summary, when it was
    # taken with the current kernel source (else null).
    from paper_1707_05354_amd import profsum
    tr = profsum.load_traffic(os.path.join(ROOT, "profiles", "paper_scale_b65536_hbm_traffic.md"))
    traffic, traffic_detail = None, None
    names = [n for n in L.KERNEL_TRACE_NAMES.get(L.KERNEL_NAMES[dom], (L.KERNEL_NAMES[dom],))
             if tr is not None and n in tr["kernels"]]
    if names:
        rows = [tr["kernels"][n] for n in names]
        disp = sum(r["dispatches"] for r in rows)
        fetch = sum(r["fetch_bytes_per_launch"] * r["dispatches"] for r in rows) / disp
        write = sum(r["write_bytes_per_launch"] * r["dispatches"] for r in rows) / disp
        traffic = round(fetch + write)
        traffic_detail = {"unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                  "copy-calibrated)",
                          "kernels": names,
                          "fetch": round(fetch),
                          "write": round(write),
                          "algorithmic": round(dom_bytes / max(1, dom_n)),
                          "traffic_over_algorithmic": round(traffic / max(1.0, dom_bytes / max(1, dom_n)), 3)}
    merge_gbs = prof.kernel_bytes[2] / max(1e-12, prof.kernel_ms[2] * 1e-3) / 1e9
    # Level merges by output size (b = 2^16: the merge into level i + 1
    # outputs 2^(i+17) elements); each line also says whether its traffic
    # (16 B per output) fits the 256 MB last-level cache.
    merge_levels = []
    lb = w.b.bit_length() - 1
    for k in range(len(prof.merge_launches_by_size)):
        n = int(prof.merge_launches_by_size[k])
        if n == 0:
            continue
        ms, byts = prof.merge_ms_by_size[k], prof.merge_bytes_by_size[k]
        merge_levels.append({"output_elems": 1 << k, "into_level": k - lb, "launches": n,
                             "avg_us": round(ms / n * 1e3, 2),
                             "GB_per_s": round(byts / (ms * 1e-3) / 1e9, 1),
                             "frac_of_hbm_peak": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "traffic_fits_mall": bool(16 * (1 << k) <= 256 * 2**20)})
    out = {
        "metric": METRIC,
        "value": round(n_upd / (upd_ms * 1e-3) / 1e6, 2),
        "unit": "M updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(float(phase.sum() / K), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "paper scale: b=2^16, %d update batches (n=%d slots, batch i deletes iff "
                        "i%%10==9), then %d lookups, %d count and %d range queries (width %d)"
                        % (w.R, n_upd, nq, nc, nr, w.width),
            "b": w.b, "batches": w.R, "key_bits": 31,
        },
        "lookups": {"value": round(nq / (lk_ms * 1e-3) / 1e6, 2), "unit": "M lookups/s",
                    "hit_rate": round(hits, 4),
                    "note": "r=1024: one occupied level (best case); see r1023"},
        "counts": {"value": round(nc / (ct_ms * 1e-3) / 1e6, 2), "unit": "M counts/s",
                   "mean_count": round(mean_count, 3)},
        "ranges": {"value": round(nr / (rg_ms * 1e-3) / 1e6, 2), "unit": "M ranges/s",
                   "pairs_returned": range_total},
        "r1023": r1023,
        "order_queries": order,
        "update_latency_ms": {"p50": round(prof.update_p50_ms, 4),
                              "p99": round(prof.update_p99_ms, 4),
                              "max": round(prof.update_max_ms, 4)},
        "phase_ms": {"updates": round(upd_ms, 3), "lookups": round(lk_ms, 3),
                     "counts": round(ct_ms, 3), "ranges": round(rg_ms, 3),
                     "sort_kernels": round(sum(prof.kernel_ms[k] for k in (0, 1, 9, 10, 11, 12)), 3),
                     "merge_kernels": round(prof.kernel_ms[2], 3),
                     "note": "sort_kernels include the cascade levels fused into the "
                             "per-bucket sorts; merge_kernels are the k_merge launches "
                             "of the levels above them"},
        "roofline": {
            "kernel": L.KERNEL_NAMES[dom],
            "bound": "hbm",
            "achieved": round(dom_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_detail": traffic_detail,
            "launches": dom_n,
            "avg_launch_us": round(dom_ms / max(1, dom_n) * 1e3, 3),
            "bytes_per_launch": round(dom_bytes / max(1, dom_n)),
            "share_of_kernel_time": round(dom_ms / max(1e-12, sum(prof.kernel_ms)), 4),
        },
        "merge_phase": {"scope": "k_merge launches only (the levels above those fused into "
                                 "the per-bucket sorts)",
                        "GB_per_s": round(merge_gbs, 1), "frac_of_hbm_peak": round(merge_gbs / HBM_PEAK_GBS, 4),
                        "by_output_size": merge_levels},
        "kernels": kernels,
        "wall_s_timed": round(wall, 3),
        "context": "paper (K40c): 98.0 M updates/s mean at b=2^16 over r=1..2048 (n=2^27); "
                   "lookups 54.9 M/s (all present) at b=2^16, n=2^24",
    }
    g.close()
    if not args.no_sweep:
        out["sweep"] = zipf_sweep(torch, L, W)
    if not args.no_batching:
        out["batching"] = batching_form(torch, L, W)
    if not args.no_serving:
        out["serving"] = serving_form(torch, L, W)
    if not args.no_cleanup:
        out["cleanup"] = cleanup_form(torch, L, W)
        out["bulk"] = bulk_form(torch, L, W)
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
