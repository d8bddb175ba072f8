"""Summaries of rocprofv3 output directories (kernel traces and PMC counters).

    python -m paper_1406_5161_amd.profsum trace DIR [--kernel SUBSTR] [--last N]
    python -m paper_1406_5161_amd.profsum pmc DIR [--kernel SUBSTR] [--last N] [--totals]
    python -m paper_1406_5161_amd.profsum traffic --fetch DIR --write DIR --calib-fetch DIR
        --calib-write DIR --calib-bytes B --kernel SUBSTR [--last N] [--source FILE ...]
        [--workload NAME] [--out JSON]

Reads either the SQLite database rocprofv3 writes by default (its `kernels` and
`pmc_events` views) or its CSV files (`*_kernel_trace.csv`,
`*_counter_collection.csv`), whichever the directory holds.  `trace` prints
calls, total, average, minimum and maximum duration per kernel, and with
--kernel the individual dispatch durations of the matching kernel (--last N:
the statistics of its last N dispatches only).  `pmc` prints, per kernel and
counter, the number of dispatches and the average value per dispatch.
With --totals, `pmc` also adds up each counter over its hardware instances (one record per
XCD or shader engine) and prints the per-dispatch totals of the --kernel dispatches.
`traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch, one run each) of a
kernel into HBM bytes per dispatch, each scaled by the factor that makes the
same counter of the calibration copy (the copy kernel with the largest value in
the calibration run, of known size B bytes) read B; the code of the --source files
(comments removed) is hashed so a reader can tell whether the kernel changed since the
counters were taken.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sqlite3
import statistics
import sys
from collections import defaultdict


def _find(d, pattern):
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def dispatches(d):
    """[(kernel name, duration ns)] in dispatch order."""
    out = []
    dbs = _find(d, "*.db")
    if dbs:
        for db in dbs:
            c = sqlite3.connect(db)
            for name, dur in c.execute("select name, duration from kernels order by start"):
                out.append((name, int(dur)))
        return out
    for f in _find(d, "*kernel_trace.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                out.append((r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return out


def counters(d):
    """[(kernel name, dispatch id, counter, value)]."""
    out = []
    dbs = _find(d, "*.db")
    if dbs:
        for db in dbs:
            c = sqlite3.connect(db)
            q = "select name, dispatch_id, counter_name, counter_value from pmc_events order by dispatch_id"
            for name, did, cn, v in c.execute(q):
                out.append((name, int(did), cn, float(v)))
        return out
    for f in _find(d, "*counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                out.append((r["Kernel_Name"], int(r["Dispatch_Id"]), r["Counter_Name"], float(r["Counter_Value"])))
    return out


def short(name, w=72):
    return name if len(name) <= w else name[: w - 3] + "..."


def cmd_trace(a):
    ds = dispatches(a.dir)
    if not ds:
        sys.exit("no kernel dispatches found under %s" % a.dir)
    by = defaultdict(list)
    for n, t in ds:
        by[n].append(t)
    total = sum(t for _, t in ds)
    print("%-72s %7s %12s %12s %12s %12s %6s" % ("kernel", "calls", "total_ms", "avg_us", "min_us", "max_us", "pct"))
    for n, ts in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        s = sum(ts)
        print("%-72s %7d %12.3f %12.2f %12.2f %12.2f %6.2f"
              % (short(n), len(ts), s * 1e-6, s * 1e-3 / len(ts), min(ts) * 1e-3, max(ts) * 1e-3, 100.0 * s / total))
    if a.kernel:
        sel = [t for n, t in ds if a.kernel in n]
        print("\ndispatches of *%s* (us): %s" % (a.kernel, " ".join("%.1f" % (t * 1e-3) for t in sel)))
        if a.last:
            sel = sel[-a.last:]
        if sel:
            print("last %d: avg %.3f us, median %.3f us, min %.3f us, max %.3f us"
                  % (len(sel), statistics.mean(sel) * 1e-3, statistics.median(sel) * 1e-3, min(sel) * 1e-3,
                     max(sel) * 1e-3))


def cmd_pmc(a):
    cs = counters(a.dir)
    if not cs:
        sys.exit("no counter records found under %s" % a.dir)
    by = defaultdict(list)
    for n, did, cn, v in cs:
        by[(n, cn)].append((did, v))
    print("%-72s %-12s %7s %16s" % ("kernel", "counter", "disp", "avg_per_disp"))
    for (n, cn), vs in sorted(by.items()):
        vals = [v for _, v in vs]
        print("%-72s %-12s %7d %16.1f" % (short(n), cn, len(vals), statistics.mean(vals)))
    if a.kernel:
        for (n, cn), vs in sorted(by.items()):
            if a.kernel not in n:
                continue
            vals = [v for _, v in sorted(vs)]
            print("\n*%s* %s per dispatch: %s" % (a.kernel, cn, " ".join("%.0f" % v for v in vals)))
            if a.last:
                vals = vals[-a.last:]
            print("last %d: avg %.1f" % (len(vals), statistics.mean(vals)))
    if a.kernel and a.totals:
        tot = defaultdict(lambda: defaultdict(float))
        inst = defaultdict(lambda: defaultdict(int))
        for n, did, cn, v in cs:
            if a.kernel in n:
                tot[cn][did] += v
                inst[cn][did] += 1
        for cn in sorted(tot):
            ds = sorted(tot[cn])
            vals = [tot[cn][d] for d in ds]
            print("\n*%s* %s total per dispatch (%d instances): %s" % (a.kernel, cn, inst[cn][ds[0]],
                                                                      " ".join("%.6g" % v for v in vals)))
            if a.last:
                vals = vals[-a.last:]
            print("last %d: avg %.6g" % (len(vals), statistics.mean(vals)))


def code_text(raw: str) -> str:
    """A C/C++/HIP source without its comments, trailing blanks and empty lines: what the
    compiler sees of it, so that editing a comment does not mark counters as stale."""
    t = re.sub(r"/\*.*?\*/", "", raw, flags=re.S)
    t = re.sub(r"//[^\n]*", "", t)
    return "\n".join(ln.rstrip() for ln in t.splitlines() if ln.strip())


def source_hash(files):
    """First 16 hex digits of SHA-256 over the code (comments removed) of the files, in order."""
    h = hashlib.sha256()
    for f in files:
        with open(f, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode("utf-8"))
    return h.hexdigest()[:16]


def _kernel_avg(d, counter, kernel, last):
    """Average over the kernel's dispatches (the last `last`) of the counter's per-dispatch total
    over its hardware instances."""
    tot = defaultdict(float)
    for n, did, cn, v in counters(d):
        if kernel in n and cn == counter:
            tot[did] += v
    vals = [tot[k] for k in sorted(tot)]
    if last:
        vals = vals[-last:]
    if not vals:
        sys.exit("no %s records of *%s* under %s" % (counter, kernel, d))
    return statistics.mean(vals), len(vals)


def _calib_kib(d, counter):
    by = defaultdict(list)
    for n, _, cn, v in counters(d):
        if cn == counter:
            by[n].append(v)
    copies = {n: v for n, v in by.items() if "copy" in n.lower()} or by
    name, vals = max(copies.items(), key=lambda kv: statistics.mean(kv[1]))
    return name, statistics.mean(vals)


def cmd_traffic(a):
    fk, nf = _kernel_avg(a.fetch, "FETCH_SIZE", a.kernel, a.last)
    wk, nw = _kernel_avg(a.write, "WRITE_SIZE", a.kernel, a.last)
    cfn, cf = _calib_kib(a.calib_fetch, "FETCH_SIZE")
    cwn, cw = _calib_kib(a.calib_write, "WRITE_SIZE")
    sf = a.calib_bytes / (cf * 1024.0)
    sw = a.calib_bytes / (cw * 1024.0)
    out = {"kernel": a.kernel, "workload": a.workload, "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
           "dispatches": [nf, nw], "calib_kernel": [cfn, cwn], "calib_bytes": a.calib_bytes,
           "calib_fetch_kib": cf, "calib_write_kib": cw, "fetch_scale": sf, "write_scale": sw,
           "hbm_bytes_per_launch": fk * 1024.0 * sf + wk * 1024.0 * sw,
           "kernel_source_sha256_16": source_hash(a.source) if a.source else None}
    text = json.dumps(out, indent=1)
    print(text)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "pmc", "traffic"])
    ap.add_argument("dir", nargs="?")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--last", type=int, default=0)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-fetch")
    ap.add_argument("--calib-write")
    ap.add_argument("--calib-bytes", type=float)
    ap.add_argument("--source", nargs="*")
    ap.add_argument("--totals", action="store_true")
    ap.add_argument("--out")
    ap.add_argument("--workload", default=None, help="name of the workload the counters were taken on")
    a = ap.parse_args()
    {"trace": cmd_trace, "pmc": cmd_pmc, "traffic": cmd_traffic}[a.mode](a)


if __name__ == "__main__":
    main()
