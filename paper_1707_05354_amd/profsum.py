"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_1707_05354_amd.profsum stats  <kernel_stats.csv>
    python -m paper_1707_05354_amd.profsum counters <fetch.csv> <write.csv> \\
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> <out.md>

    python -m paper_1707_05354_amd.profsum readsizes <sizes.csv> <copy_sizes.csv> \
        <copy_bytes> <traffic.md> <out.md>

`counters` scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what the same
counters read for a plain device copy of copy_bytes bytes, and writes a
Markdown summary whose `traffic-json:` line bench.py reads back.  The line
records the SHA-256 of the kernel source the counters were taken with; when
the source has changed since, bench.py reports traffic as null.

`readsizes` checks that scale per kernel.  FETCH_SIZE weighs the L2's read
requests to memory by their size, and one scale taken from a streaming copy
is exact only for kernels whose requests have the copy's size mix.  The
gfx950 L2 also counts its 32-, 64- and 128-byte read requests separately
(TCC_EA0_RDREQ_32B/64B/128B); their byte sum is the read traffic with no
scale at all, and the summary sets it beside the scaled FETCH_SIZE of the
traffic summary for every kernel.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "lsm_kernels.hip")


def kernel_source_sha256() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short_name(n: str) -> str:
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"lsm::\(anonymous namespace\)::", "", n)
    m = re.match(r"([A-Za-z_0-9:]+(?:<[^>]*>)?)\(", n)
    return (m.group(1) if m else n)[:60]


def stats(path: str):
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]),
                     float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"]),
                     float(r["Percentage"])))
    return rows


def counter_means(path: str):
    """kernel -> (dispatches, mean KiB per dispatch)."""
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(path)):
        k = short_name(r["Kernel_Name"])
        agg[k][0] += 1
        agg[k][1] += float(r["Counter_Value"])
    return {k: (n, v / n) for k, (n, v) in agg.items()}


def copy_kib(path: str) -> float:
    """Mean counter value of the largest device-copy dispatches."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if "copy" in r["Kernel_Name"].lower()]
    top = max(vals)
    return sum(v for v in vals if v > 0.5 * top) / len([v for v in vals if v > 0.5 * top])


def counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, out_md, command):
    f, w = counter_means(fetch_csv), counter_means(write_csv)
    cf, cw = copy_kib(copy_fetch_csv), copy_kib(copy_write_csv)
    fscale = copy_bytes / (cf * 1024.0)
    wscale = copy_bytes / (cw * 1024.0)
    table = {}
    for k in sorted(set(f) | set(w)):
        if k not in f or k not in w:
            continue
        table[k] = {"dispatches": f[k][0],
                    "fetch_bytes_per_launch": f[k][1] * 1024.0 * fscale,
                    "write_bytes_per_launch": w[k][1] * 1024.0 * wscale}
    doc = {"kernel_source_sha256": kernel_source_sha256(), "fetch_scale": fscale,
           "write_scale": wscale, "kernels": table}
    lines = ["# HBM traffic per kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a plain copy)", "",
             "Commands (from the repository root):", "", "```"] + command + ["```", "",
             "Copy calibration: %d bytes read and written; FETCH_SIZE reads %.1f KiB (scale %.3f), "
             "WRITE_SIZE reads %.1f KiB (scale %.3f)." % (copy_bytes, cf, fscale, cw, wscale), "",
             "| kernel | dispatches | fetch bytes / launch | write bytes / launch |", "|---|---|---|---|"]
    for k, v in table.items():
        lines.append("| %s | %d | %.0f | %.0f |" % (k, v["dispatches"], v["fetch_bytes_per_launch"],
                                                   v["write_bytes_per_launch"]))
    lines += ["", "traffic-json: " + json.dumps(doc, sort_keys=True), ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    return doc


SIZE_COUNTERS = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64),
                 ("TCC_EA0_RDREQ_128B_sum", 128))


def request_sizes(path: str):
    """kernel -> (dispatches, mean 32/64/128-byte read requests per dispatch)."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in csv.DictReader(open(path)):
        d = r["Dispatch_Id"]
        names[d] = short_name(r["Kernel_Name"])
        per[d][r["Counter_Name"]] += float(r["Counter_Value"])
    agg = collections.defaultdict(lambda: [0, [0.0, 0.0, 0.0]])
    for d, c in per.items():
        a = agg[names[d]]
        a[0] += 1
        for i, (name, _) in enumerate(SIZE_COUNTERS):
            a[1][i] += c.get(name, 0.0)
    return {k: (n, [v / n for v in t]) for k, (n, t) in agg.items()}


def request_bytes(reqs) -> float:
    return sum(n * size for n, (_, size) in zip(reqs, SIZE_COUNTERS))


def readsizes(sizes_csv, copy_csv, copy_bytes, traffic_md, out_md, command):
    sz = request_sizes(sizes_csv)
    cp = request_sizes(copy_csv)
    copy_rows = [(k, v) for k, v in cp.items() if "copy" in k.lower()]
    copy_read = max(request_bytes(v[1]) for _, v in copy_rows)
    traffic = load_traffic(traffic_md)
    scaled = traffic["kernels"] if traffic else {}
    rows = {}
    for k, (n, reqs) in sorted(sz.items()):
        b = request_bytes(reqs)
        f = scaled.get(k, {}).get("fetch_bytes_per_launch")
        rows[k] = {"dispatches": n, "req32": reqs[0], "req64": reqs[1], "req128": reqs[2],
                   "read_bytes_per_launch": b, "scaled_fetch_bytes_per_launch": f,
                   "scaled_over_sized": (f / b) if (f and b > 0) else None}
    doc = {"kernel_source_sha256": kernel_source_sha256(), "copy_bytes": copy_bytes,
           "copy_read_bytes_from_sizes": copy_read, "kernels": rows}
    lines = ["# Read traffic per kernel from the L2's request sizes (rocprofv3, gfx950)", "",
             "Bytes read from memory per launch = 32 x TCC_EA0_RDREQ_32B_sum + 64 x "
             "TCC_EA0_RDREQ_64B_sum + 128 x TCC_EA0_RDREQ_128B_sum, with no calibration "
             "factor, beside the copy-scaled FETCH_SIZE figure of the traffic summary of the "
             "same kernel source (ratio 1 when the scale is right for that kernel).", "",
             "Commands (from the repository root):", "", "```"] + command + ["```", "",
             "Plain device copy: %d bytes read; the request sizes give %.0f bytes (%.4f)."
             % (copy_bytes, copy_read, copy_read / copy_bytes), "",
             "| kernel | dispatches | 32 B req | 64 B req | 128 B req | read bytes / launch "
             "| scaled FETCH_SIZE / launch | scaled / sized |", "|---|---|---|---|---|---|---|---|"]
    for k, v in rows.items():
        lines.append("| %s | %d | %.0f | %.0f | %.0f | %.0f | %s | %s |" % (
            k, v["dispatches"], v["req32"], v["req64"], v["req128"], v["read_bytes_per_launch"],
            "%.0f" % v["scaled_fetch_bytes_per_launch"] if v["scaled_fetch_bytes_per_launch"] else "-",
            "%.3f" % v["scaled_over_sized"] if v["scaled_over_sized"] else "-"))
    lines += ["", "readsizes-json: " + json.dumps(doc, sort_keys=True), ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    return doc


def load_traffic(md_path: str):
    """The traffic table of a summary, or None when missing or stale."""
    if not os.path.exists(md_path):
        return None
    for line in open(md_path):
        if line.startswith("traffic-json: "):
            doc = json.loads(line[len("traffic-json: "):])
            if doc.get("kernel_source_sha256") != kernel_source_sha256():
                return None
            return doc
    return None


def main(argv):
    if argv[0] == "stats":
        for s in stats(argv[1]):
            print("%-44s calls=%7d total_ms=%9.3f avg_us=%9.3f min_us=%8.3f max_us=%9.3f pct=%6.2f"
                  % (s[0], s[1], s[2] / 1e6, s[3] / 1e3, s[4] / 1e3, s[5] / 1e3, s[6]))
    elif argv[0] == "counters":
        cmd = os.environ.get("PROFSUM_COMMANDS", "").split(";;")
        doc = counters(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6], [c for c in cmd if c])
        print(json.dumps(doc, indent=1))
    elif argv[0] == "readsizes":
        cmd = os.environ.get("PROFSUM_COMMANDS", "").split(";;")
        doc = readsizes(argv[1], argv[2], int(argv[3]), argv[4], argv[5], [c for c in cmd if c])
        print(json.dumps(doc, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
