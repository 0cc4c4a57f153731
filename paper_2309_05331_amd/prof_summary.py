"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2309_05331_amd.prof_summary kernel-trace RESULTS.db [--min-us 20]
    python -m paper_2309_05331_amd.prof_summary counters FETCH.csv WRITE.csv [--fetch-scale 2] [--write-scale 1]

kernel-trace: per-kernel dispatch count, mean/min/max duration over real
dispatches only.  The integration loop launches graph chunks whose kernels
return at once after the run has finished; those empty launches (shorter than
--min-us) are counted separately instead of diluting the mean.

counters: per-kernel mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from
two rocprofv3 --pmc runs, scaled by the factors the reference copy kernel
establishes (what the counter reads for a known byte count), and the HBM
bytes per dispatch.
"""
from __future__ import annotations

import argparse
import collections
import csv
import re
import sqlite3


def short(name: str) -> str:
    m = re.search(r"gs_stage<(\w+), (\d+), (\d+), (\d+)>", name)
    if m:
        kinds = ["D1", "R2", "R3", "R4", "D2", "D3", "D4", "D5", "D6", "D7", "D7F", "D6F"]
        return "gs_stage %s %s ry=%s vw=%s" % (kinds[int(m.group(2))], m.group(1), m.group(3), m.group(4))
    m = re.search(r"(\w+)\(", name)
    return (m.group(1) if m else name)[:60]


def kernel_trace(db: str, min_us: float):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, start, end from kernels"))
    agg = collections.defaultdict(list)
    empty = collections.Counter()
    for name, s, e in rows:
        us = (e - s) / 1e3
        if us < min_us:
            empty[short(name)] += 1
        else:
            agg[short(name)].append(us)
    lines = ["%-40s %8s %12s %12s %12s %8s" % ("kernel", "calls", "mean_us", "min_us", "max_us", "empty")]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append("%-40s %8d %12.2f %12.2f %12.2f %8d" % (k, len(v), sum(v) / len(v), min(v), max(v), empty[k]))
    for k, n in empty.items():
        if k not in agg:
            lines.append("%-40s %8d %12s %12s %12s %8d" % (k, 0, "-", "-", "-", n))
    return "\n".join(lines)


def counters(fetch_csv: str, write_csv: str, fs: float, ws: float):
    def load(path, cname):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == cname:
                agg[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return agg
    f = load(fetch_csv, "FETCH_SIZE")
    w = load(write_csv, "WRITE_SIZE")
    lines = ["%-40s %6s %14s %14s %16s" % ("kernel", "n", "FETCH_KiB", "WRITE_KiB", "HBM_bytes_scaled")]
    for k in sorted(set(f) | set(w)):
        fm = sum(f[k]) / len(f[k]) if f.get(k) else 0.0
        wm = sum(w[k]) / len(w[k]) if w.get(k) else 0.0
        lines.append("%-40s %6d %14.1f %14.1f %16.4g" % (k, max(len(f.get(k, [])), len(w.get(k, []))), fm, wm,
                                                        (fm * fs + wm * ws) * 1024))
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernel-trace")
    a.add_argument("db")
    a.add_argument("--min-us", type=float, default=20.0)
    b = sub.add_parser("counters")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--fetch-scale", type=float, default=2.0)
    b.add_argument("--write-scale", type=float, default=1.0)
    args = ap.parse_args()
    if args.cmd == "kernel-trace":
        print(kernel_trace(args.db, args.min_us))
    else:
        print(counters(args.fetch_csv, args.write_csv, args.fetch_scale, args.write_scale))


if __name__ == "__main__":
    main()
