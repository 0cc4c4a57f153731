"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2309_05331_amd.prof_summary kernel-trace RESULTS.db [--min-us 20]
    python -m paper_2309_05331_amd.prof_summary counters FETCH.csv WRITE.csv [--fetch-scale 2] [--write-scale 1]
    python -m paper_2309_05331_amd.prof_summary counters-json FETCH.csv WRITE.csv --kernel NAME --tag TAG --workload W

kernel-trace: per-kernel dispatch count, mean/min/max duration over real
dispatches only.  The integration loop launches graph chunks whose kernels
return at once after the run has finished; those empty launches (shorter than
--min-us, or than 5% of the median of the kernel's longer launches) are counted
separately instead of diluting the mean.

counters: per-kernel mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch, real
dispatches only, as above) from two rocprofv3 --pmc runs, scaled by the factors the reference copy kernel
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
    m = re.search(r"gs_stage<(\w+), (\d+), (\d+), (\d+)(?:, (\d+))?>", name)
    if m:
        kinds = (["D1", "R2", "R3", "R4", "D2", "D3", "D4", "D5", "D6", "D7", "D7F", "C4", "C5", "C6", "C6F", "E1",
                  "D6F"] + ["F%d" % i for i in range(1, 14)] + ["F13F"] + ["AB%d" % s for s in range(1, 9)] + ["D6K"] + ["ABC%d" % s for s in range(1, 9)] + ["MM1", "MM2", "MM3"])
        nw = " nw=%s" % m.group(5) if m.group(5) and m.group(5) != "4" else ""
        return "gs_stage %s %s ry=%s vw=%s%s" % (kinds[int(m.group(2))], m.group(1), m.group(3), m.group(4), nw)
    m = re.search(r"(ew_\w+)<(\w+), (\d+)(?:, (\d+))?", name)
    if m:
        third = "" if not m.group(4) else (" mode=%s" if m.group(1) == "ew_step" else " s=%s") % m.group(4)
        return "%s %s rhs=%s%s" % (m.group(1), m.group(2), m.group(3), third)
    m = re.search(r"ens_kernel<(\w+)>", name)
    if m:
        return "ens_kernel %s" % m.group(1)
    m = re.search(r"(\w+)\(", name)
    return (m.group(1) if m else name)[:60]


EMPTY_FRAC = 0.05


def _split_empty(durations, min_us):
    """Flags of the dispatches that did work: at least min_us long and at
    least EMPTY_FRAC of the median of the kernel's dispatches that are."""
    longer = sorted(d for d in durations if d >= min_us)
    cut = max(min_us, EMPTY_FRAC * longer[len(longer) // 2]) if longer else min_us
    return [d >= cut for d in durations]


def kernel_trace(db: str, min_us: float):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, start, end from kernels"))
    per = collections.defaultdict(list)
    for name, s, e in rows:
        per[short(name)].append((e - s) / 1e3)
    agg = collections.defaultdict(list)
    empty = collections.Counter()
    for k, ds in per.items():
        for d, real in zip(ds, _split_empty(ds, min_us)):
            if real:
                agg[k].append(d)
            else:
                empty[k] += 1
    lines = ["%-40s %8s %12s %12s %12s %8s" % ("kernel", "calls", "mean_us", "min_us", "max_us", "empty")]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append("%-40s %8d %12.2f %12.2f %12.2f %8d" % (k, len(v), sum(v) / len(v), min(v), max(v), empty[k]))
    for k, n in empty.items():
        if k not in agg:
            lines.append("%-40s %8d %12s %12s %12s %8d" % (k, 0, "-", "-", "-", n))
    return "\n".join(lines)


def _load(path, cname, min_us=20.0):
    """Counter values per kernel over real dispatches only: graph-chunk
    launches that return at once are left out by the kernel trace's rule, so
    they do not dilute the per-dispatch means."""
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != cname:
            continue
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        per[short(r["Kernel_Name"])].append((us, float(r["Counter_Value"])))
    agg = collections.defaultdict(list)
    for k, rows in per.items():
        for (_, v), real in zip(rows, _split_empty([us for us, _ in rows], min_us)):
            if real:
                agg[k].append(v)
    return agg


def counters_record(fetch_csv, write_csv, fs, ws, kernel, tag, workload, source, per="launch", min_us=20.0):
    """JSON record of one kernel's mean scaled HBM bytes per dispatch (or the
    sum over all its dispatches with per="run"), stamped with the SHA-256 of
    the kernel's source files (concatenated in the order given) so a reader
    can tell whether it still applies."""
    import hashlib
    import os
    f = _load(fetch_csv, "FETCH_SIZE", min_us)[kernel]
    w = _load(write_csv, "WRITE_SIZE", min_us)[kernel]
    if not f or not w:
        raise SystemExit("kernel %r not in the counter files" % kernel)
    agg = (lambda v: sum(v)) if per == "run" else (lambda v: sum(v) / len(v))
    fk, wk = agg(f), agg(w)
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    names = [x for x in source.split(",") if x]
    h = hashlib.sha256()
    for nm in names:
        h.update(open(os.path.join(here, nm), "rb").read())
    return {"kernel": tag, "workload": workload, "sources": names, "sources_sha256": h.hexdigest(),
            "fetch_kib": round(fk, 1), "write_kib": round(wk, 1), "fetch_scale": fs, "write_scale": ws,
            "dispatches": len(f), "per": per,
            "hbm_bytes_per_launch" if per == "launch" else "hbm_bytes_per_run": int(round((fk * fs + wk * ws) * 1024))}


def counters(fetch_csv: str, write_csv: str, fs: float, ws: float, min_us: float = 20.0):
    f = _load(fetch_csv, "FETCH_SIZE", min_us)
    w = _load(write_csv, "WRITE_SIZE", min_us)
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
    b.add_argument("--min-us", type=float, default=20.0)
    j = sub.add_parser("counters-json")
    j.add_argument("fetch_csv")
    j.add_argument("write_csv")
    j.add_argument("--kernel", required=True, help="summary name of the kernel, e.g. 'gs_stage D6 float ry=1 vw=4'")
    j.add_argument("--tag", required=True, help="short kernel tag used by bench.py, e.g. D6")
    j.add_argument("--workload", required=True)
    j.add_argument("--source", default="stage.h,gs.hip,hode_dev.h,hode_internal.h",
                   help="comma-separated kernel sources and the headers they include, under csrc/")
    j.add_argument("--per", choices=["launch", "run"], default="launch")
    j.add_argument("--fetch-scale", type=float, default=2.0)
    j.add_argument("--write-scale", type=float, default=1.0)
    j.add_argument("--min-us", type=float, default=20.0)
    args = ap.parse_args()
    if args.cmd == "kernel-trace":
        print(kernel_trace(args.db, args.min_us))
    elif args.cmd == "counters":
        print(counters(args.fetch_csv, args.write_csv, args.fetch_scale, args.write_scale, args.min_us))
    else:
        import json
        print(json.dumps(counters_record(args.fetch_csv, args.write_csv, args.fetch_scale, args.write_scale,
                                         args.kernel, args.tag, args.workload, args.source, args.per,
                                         args.min_us), indent=1))


if __name__ == "__main__":
    main()
