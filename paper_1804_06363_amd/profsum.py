"""Summaries of rocprofv3 CSV output (kernel statistics and PMC counters) as short text.

    python -m paper_1804_06363_amd.profsum stats DIR            # *kernel_stats.csv
    python -m paper_1804_06363_amd.profsum counters DIR NAME    # *counter_collection.csv

`counters` aggregates one counter per kernel name: dispatches, mean and total value.
"""
from __future__ import annotations

import csv
import glob
import os
import sys
from collections import defaultdict


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits


def _short(name, width=90):
    name = name.replace("void ", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(d):
    rows = []
    for path in _find(d, "*kernel_stats.csv"):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    print(f"{'calls':>7} {'total ms':>10} {'avg us':>10}  kernel")
    for r in rows[:40]:
        calls = int(r["Calls"])
        tot = float(r["TotalDurationNs"]) / 1e6
        avg = float(r["AverageNs"]) / 1e3
        print(f"{calls:7d} {tot:10.3f} {avg:10.1f}  {_short(r['Name'])}")


def counters(d, name):
    agg = defaultdict(lambda: [0, 0.0])
    for path in _find(d, "*counter_collection.csv"):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != name:
                    continue
                a = agg[r["Kernel_Name"]]
                a[0] += 1
                a[1] += float(r["Counter_Value"])
    print(f"counter {name}")
    print(f"{'dispatches':>10} {'mean/dispatch':>16} {'total':>16}  kernel")
    for k, (n, tot) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:40]:
        print(f"{n:10d} {tot / n:16.1f} {tot:16.1f}  {_short(k)}")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
