"""Summaries of rocprofv3 CSV output (kernel statistics and PMC counters) as short text.

    python -m paper_1804_06363_amd.profsum stats DIR            # *kernel_stats.csv
    python -m paper_1804_06363_amd.profsum counters DIR NAME    # *counter_collection.csv
    python -m paper_1804_06363_amd.profsum gaps DIR NAME COUNT [LAST]  # *kernel_trace.csv

`counters` aggregates one counter per kernel name: dispatches, mean and total value.
`gaps` splits a kernel trace by stream, from the earliest of the last COUNT dispatches of
kernels whose name contains NAME on: per stream the span from its first kernel start to
its last kernel end (or to the end of its last kernel whose name contains LAST), the time
covered by its kernels, the share of the span when none of its kernels ran (launch gaps
and host waits) and the median gap between consecutive kernels, with its most frequent
kernel.
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


def gaps(d, name, count, last=None):
    rows = []
    for path in _find(d, "*kernel_trace.csv"):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    key = "Stream_Id" if rows and "Stream_Id" in rows[0] else "Queue_Id"
    marks = sorted(int(r["Start_Timestamp"]) for r in rows if name in r["Kernel_Name"])
    if len(marks) < count:
        raise SystemExit(f"fewer than {count} dispatches of {name}")
    t0 = marks[-count]
    streams = defaultdict(list)
    for r in rows:
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if a >= t0:
            streams[r[key]].append((a, b, r["Kernel_Name"]))
    print(f"window from the last {count} dispatches of {name}; per {key}")
    print(f"{'stream':>8} {'kernels':>8} {'span ms':>10} {'busy ms':>10} {'gap share':>10}"
          f" {'median gap us':>14}  most frequent kernel (mean us)")
    for sid, ks in sorted(streams.items(), key=lambda kv: -len(kv[1])):
        ks.sort()
        if last:
            ends = [i for i, (_, _, n) in enumerate(ks) if last in n]
            if ends:
                ks = ks[:ends[-1] + 1]
        gl = sorted(max(0, ks[i + 1][0] - ks[i][1]) for i in range(len(ks) - 1)) or [0]
        busy, cur_a, cur_b = 0, None, None
        for a, b, _ in ks:  # union of the kernel intervals
            if cur_b is None or a > cur_b:
                if cur_b is not None:
                    busy += cur_b - cur_a
                cur_a, cur_b = a, b
            else:
                cur_b = max(cur_b, b)
        busy += cur_b - cur_a
        span = max(b for _, b, _ in ks) - ks[0][0]
        freq = defaultdict(list)
        for a, b, n in ks:
            freq[n].append(b - a)
        top, durs = max(freq.items(), key=lambda kv: len(kv[1]))
        print(f"{sid:>8} {len(ks):8d} {span / 1e6:10.2f} {busy / 1e6:10.2f} "
              f"{1 - busy / max(span, 1):10.3f} {gl[len(gl) // 2] / 1e3:14.1f}  "
              f"{_short(top, 60)} ({sum(durs) / len(durs) / 1e3:.1f})")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 5 and sys.argv[1] == "gaps":
        gaps(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5] if len(sys.argv) > 5 else None)
    else:
        raise SystemExit(__doc__)
