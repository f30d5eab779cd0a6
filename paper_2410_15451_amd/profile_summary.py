#!/usr/bin/env python3
"""Summaries of rocprofv3 CSV output for the Leiden library.

kernels DIR [--between REGEX] [--window K] [--top N]
    Per-kernel dispatch count, total and average duration from the kernel
    trace under DIR.  With --between, only the dispatches strictly between
    marker dispatches 2K and 2K + 1 (those whose name matches REGEX) are
    counted: bench.py --marker launches a marker kernel right before and
    right after its timed static run (window 0) and its timed update steps
    (window 1).

counters FETCH_DIR WRITE_DIR --kernel NAME --calib-bytes B [--between REGEX] [--window K] [--steps S]
    Average FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the kernel whose
    name starts with NAME, each scaled by what the same counter reads for the
    first device copy of the run (bench.py's calibration copy of B bytes,
    which reads and writes B bytes), and the resulting HBM bytes per launch
    as JSON.  NAME '*' sums every dispatch of the window instead and reports
    the HBM bytes per step (the window holding S steps).

Reads only rocprofv3's CSV files (--output-format csv).
"""
import argparse
import csv
import glob
import json
import os
import re
import sys


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        sys.exit("no *%s under %s" % (suffix, d))
    return hits[0]


def _col(header, *names):
    low = [h.lower() for h in header]
    for n in names:
        if n.lower() in low:
            return low.index(n.lower())
    sys.exit("none of %s in CSV header %s" % (names, header))


def _short(name):
    return re.sub(r"\(.*", "", name).strip()


WINDOW = 0  # which pair of marker dispatches bounds the window (--window)


def _window(names, between):
    """Index range (lo, hi) of the dispatches between marker dispatches
    2K and 2K + 1 (K = --window), or the whole list."""
    if not between:
        return 0, len(names)
    rx = re.compile(between)
    marks = [i for i, nm in enumerate(names) if rx.search(nm)]
    if len(marks) < 2 * WINDOW + 2:
        sys.exit("fewer than %d dispatches match %r" % (2 * WINDOW + 2, between))
    return marks[2 * WINDOW] + 1, marks[2 * WINDOW + 1]


def kernels(args):
    path = _find(args.dir, "kernel_trace.csv")
    with open(path, newline="") as f:
        rd = csv.reader(f)
        hdr = next(rd)
        ni = _col(hdr, "Kernel_Name")
        si = _col(hdr, "Start_Timestamp")
        ei = _col(hdr, "End_Timestamp")
        rows = sorted(((int(r[si]), int(r[ei]), r[ni]) for r in rd), key=lambda t: t[0])
    lo, hi = _window([r[2] for r in rows], args.between)
    agg = {}
    for s, e, nm in rows[lo:hi]:
        a = agg.setdefault(_short(nm), [0, 0])
        a[0] += 1
        a[1] += e - s
    busy = sum(v[1] for v in agg.values())
    span = (rows[hi - 1][1] - rows[lo][0]) if hi > lo else 0
    print("dispatches %d, kernel-busy %.3f ms over a span of %.3f ms" % (hi - lo, busy / 1e6, span / 1e6))
    print("%10s %7s %7s %11s  %s" % ("total_ms", "share", "calls", "avg_us", "kernel"))
    for nm, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:args.top]:
        print("%10.3f %6.1f%% %7d %11.1f  %s" % (t / 1e6, 100.0 * t / max(busy, 1), c, t / c / 1e3, nm))


def _counter_rows(d, counter):
    path = _find(d, "counter_collection.csv")
    with open(path, newline="") as f:
        rd = csv.reader(f)
        hdr = next(rd)
        di = _col(hdr, "Dispatch_Id", "Correlation_Id")
        ni = _col(hdr, "Kernel_Name")
        ci = _col(hdr, "Counter_Name")
        vi = _col(hdr, "Counter_Value")
        per = {}
        for r in rd:
            if r[ci] != counter:
                continue
            k = int(r[di])
            nm, v = per.get(k, (r[ni], 0.0))
            per[k] = (nm, v + float(r[vi]))
    return [(k, nm, v) for k, (nm, v) in sorted(per.items())]


def _kernel_avg(rows, prefix, between):
    lo, hi = _window([r[1] for r in rows], between)
    vals = [v for _, nm, v in rows[lo:hi] if _short(nm).startswith(prefix)]
    if not vals:
        sys.exit("no dispatch of %r" % prefix)
    return sum(vals) / len(vals), len(vals)


def _copy_factor(rows, calib_bytes):
    """bench.py --calib-copy-mib launches its device copy before any other
    copy of the run: the first copy dispatch is the calibration copy."""
    copies = [v for _, nm, v in rows if "copyBuffer" in nm]
    if not copies or copies[0] <= 0:
        sys.exit("no copy dispatch for calibration")
    return (calib_bytes / 1024.0) / copies[0]


def _window_sum(rows, between):
    lo, hi = _window([r[1] for r in rows], between)
    return sum(v for _, _, v in rows[lo:hi]), hi - lo


def counters(args):
    fr = _counter_rows(args.fetch_dir, "FETCH_SIZE")
    wr = _counter_rows(args.write_dir, "WRITE_SIZE")
    ff, fw = _copy_factor(fr, args.calib_bytes), _copy_factor(wr, args.calib_bytes)
    if args.kernel == "*":
        fs, fn = _window_sum(fr, args.between)
        ws, wn = _window_sum(wr, args.between)
        out = {"kernel": "*", "steps": args.steps, "fetch_kib_per_step": fs / args.steps,
               "write_kib_per_step": ws / args.steps, "fetch_factor": ff, "write_factor": fw,
               "dispatches_fetch_run": fn, "dispatches_write_run": wn,
               "hbm_bytes_per_step": (fs * ff + ws * fw) * 1024.0 / args.steps}
        print(json.dumps(out, indent=1))
        return
    fk, fn = _kernel_avg(fr, args.kernel, args.between)
    wk, wn = _kernel_avg(wr, args.kernel, args.between)
    out = {"kernel": args.kernel, "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
           "fetch_factor": ff, "write_factor": fw, "launches_fetch_run": fn, "launches_write_run": wn,
           "hbm_bytes_per_launch": (fk * ff + wk * fw) * 1024.0}
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("dir")
    k.add_argument("--between", default="")
    k.add_argument("--top", type=int, default=25)
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--steps", type=int, default=1)
    c.add_argument("--calib-bytes", type=float, required=True)
    c.add_argument("--between", default="")
    for p in (k, c):
        p.add_argument("--window", type=int, default=0,
                       help="marker pair bounding the window (bench.py --marker: 0 = the timed static run, "
                            "1 = the timed update steps)")
    a = ap.parse_args()
    global WINDOW
    WINDOW = a.window
    (kernels if a.cmd == "kernels" else counters)(a)


if __name__ == "__main__":
    main()
