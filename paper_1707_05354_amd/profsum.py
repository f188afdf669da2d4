"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_1707_05354_amd.profsum stats  <kernel_stats.csv>
    python -m paper_1707_05354_amd.profsum counters <fetch.csv> <write.csv> \\
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> <out.md>

`counters` scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what the same
counters read for a plain device copy of copy_bytes bytes, and writes a
Markdown summary whose `traffic-json:` line bench.py reads back.  The line
records the SHA-256 of the kernel source the counters were taken with; when
the source has changed since, bench.py reports traffic as null.
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
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
