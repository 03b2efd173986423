"""Summaries of rocprofv3 CSV output for the filter kernels.

    python -m paper_2006_08498_amd.profsum stats DIR [--match SUBSTR]
    python -m paper_2006_08498_amd.profsum traffic --fetch D --write D \
        --copy-fetch D --copy-write D --copy-bytes B [--match SUBSTR] [--workload W]
    python -m paper_2006_08498_amd.profsum counters DIR [--match SUBSTR]
    python -m paper_2006_08498_amd.profsum trace DIR [--match SUBSTR] [--last K]
    python -m paper_2006_08498_amd.profsum bandwidth --trace D --fetch D --write D \
        --copy-fetch D --copy-write D --copy-bytes B [--match A,B,...]

`stats` prints the rows of the kernel-statistics CSV under DIR (from
`rocprofv3 --kernel-trace --stats --output-format csv`) whose kernel name
contains SUBSTR, plus their call-weighted average duration.

`trace` prints each matching kernel's average dispatch duration from a
kernel trace (`--kernel-trace --output-format csv`); `--last K` keeps each
kernel's last K dispatches only (here and in `traffic`), which singles out
the launches a benchmark times when the same kernel also ran before them.

`counters` prints, per kernel, the mean per dispatch of every counter of
a `--pmc` run (for instance MfmaUtil, the percentage of cycles the MFMA
units were busy).

`bandwidth` joins a kernel trace with the two counter runs: per kernel,
the average duration and the calibrated HBM bytes per dispatch, hence the
achieved bandwidth against the HBM peak (8 TB/s).

`traffic` turns two counter runs (`--pmc FETCH_SIZE`, then `--pmc
WRITE_SIZE`, KiB per dispatch) into HBM bytes per launch.  Each counter is
scaled by the factor that maps what it reads for a plain device copy of B
bytes (read B, write B) to B, so the figures are in true bytes whatever
fraction of the memory channels the counter observes.  The last line is a
JSON record, prefixed `traffic-record:`, that carries the digest of the
kernel sources it was measured on; a benchmark reports the traffic only
while the digest still matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# Sources that define each filter kernel and its launch plan.
KERNEL_SOURCES = {
    "k_filter": ("k_filter_kern.h", "k_filter.hip", "k_filter_wide.hip", "k_filter_plan.h"),
    "k_filter32": ("k_filter32.hip", "k_filter_plan.h"),
    "k_ingest_rows": ("k_ingest.hip",),
    "k_herm_complete": ("k_ingest.hip",),
}


def sources_digest(kernel: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _csvs(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def kernel_stats(d, match):
    rows = []
    for f in _csvs(d, "kernel_stats.csv"):
        for r in csv.DictReader(open(f)):
            if match in r["Name"]:
                rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]),
                             float(r["TotalDurationNs"])))
    return rows


def counter_values(d, match, counter, last=0):
    """Per-dispatch values of `counter` for kernels whose name contains match
    (with last > 0: only each kernel's last `last` dispatches, by dispatch
    id)."""
    per = collections.defaultdict(list)
    for f in _csvs(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
                per[r["Kernel_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    out = {}
    for name, v in per.items():
        v.sort()
        out[name] = [x for _, x in (v[-last:] if last > 0 else v)]
    return out


def trace_durations(d, match, last=0):
    """Per-dispatch durations (ns) from a kernel trace, per kernel name, in
    dispatch order (with last > 0: each kernel's last `last` dispatches)."""
    per = collections.defaultdict(list)
    for f in _csvs(d, "kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            if match in r["Kernel_Name"]:
                per[r["Kernel_Name"]].append(
                    (int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = {}
    for name, v in per.items():
        v.sort()
        out[name] = [x for _, x in (v[-last:] if last > 0 else v)]
    return out


def _short(name):
    # 'void ns::(anonymous namespace)::k_filter<9, 0, false>(args...)'
    #   -> 'k_filter<9, 0, false>'
    head = name.replace("(anonymous namespace)", "anon").split("(")[0]
    return head.replace("void ", "").split("::")[-1]


def cmd_stats(a):
    rows = kernel_stats(a.dir, a.match)
    calls = sum(r[1] for r in rows)
    total = sum(r[3] for r in rows)
    print("| kernel | calls | avg us | total ms |")
    print("|---|---:|---:|---:|")
    for name, c, avg, tot in sorted(rows, key=lambda r: -r[3]):
        print(f"| {_short(name)} | {c} | {avg / 1e3:.2f} | {tot / 1e6:.2f} |")
    if calls:
        print(f"| all `{a.match}` | {calls} | {total / calls / 1e3:.2f} | {total / 1e6:.2f} |")


def cmd_traffic(a):
    cf = counter_values(a.copy_fetch, "copy", "FETCH_SIZE")
    cw = counter_values(a.copy_write, "copy", "WRITE_SIZE")
    cf_mean = sum(sum(v) for v in cf.values()) / max(1, sum(len(v) for v in cf.values()))
    cw_mean = sum(sum(v) for v in cw.values()) / max(1, sum(len(v) for v in cw.values()))
    if cf_mean <= 0 or cw_mean <= 0:
        sys.exit("copy-kernel counters missing")
    kf = a.copy_bytes / (cf_mean * 1024.0)
    kw = a.copy_bytes / (cw_mean * 1024.0)
    fv = counter_values(a.fetch, a.match, "FETCH_SIZE", a.last)
    wv = counter_values(a.write, a.match, "WRITE_SIZE", a.last)
    print(f"copy of {a.copy_bytes} bytes: FETCH_SIZE {cf_mean:.6g} KiB -> factor {kf:.4f}; "
          f"WRITE_SIZE {cw_mean:.6g} KiB -> factor {kw:.4f}")
    print()
    print("| kernel | launches | read GB/launch | written MB/launch |")
    print("|---|---:|---:|---:|")
    nf = nw = 0
    sf = sw = 0.0
    for name in sorted(fv):
        f = fv[name]
        w = wv.get(name, [])
        nf += len(f)
        nw += len(w)
        sf += sum(f)
        sw += sum(w)
        rd = kf * 1024.0 * sum(f) / len(f)
        wr = kw * 1024.0 * sum(w) / max(1, len(w))
        print(f"| {_short(name)} | {len(f)} | {rd / 1e9:.3f} | {wr / 1e6:.2f} |")
    if nf == 0 or nw == 0:
        sys.exit("kernel counters missing")
    rd = kf * 1024.0 * sf / nf
    wr = kw * 1024.0 * sw / nw
    print(f"| all | {nf} | {rd / 1e9:.3f} | {wr / 1e6:.2f} |")
    print()
    kern = a.kernel or ("k_filter32" if "k_filter32" in a.match else "k_filter")
    rec = {"kernel": kern, "workload": a.workload, "sources_digest": sources_digest(kern),
           "launches": nf, "read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
           "bytes_per_launch": rd + wr, "fetch_factor": kf, "write_factor": kw}
    print("traffic-record: " + json.dumps(rec))


def cmd_trace(a):
    """Average duration of each matching kernel's dispatches in a trace."""
    print("| kernel | dispatches | avg us | min us | max us |")
    print("|---|---:|---:|---:|---:|")
    for name, v in sorted(trace_durations(a.dir, a.match, a.last).items()):
        print(f"| {_short(name)} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | "
              f"{min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} |")


def cmd_counters(a):
    """Mean per dispatch of every counter in the run, per kernel width."""
    names = collections.defaultdict(dict)
    for f in _csvs(a.dir, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            if a.match in r["Kernel_Name"]:
                d = names[_short(r["Kernel_Name"])].setdefault(r["Counter_Name"], [])
                d.append(float(r["Counter_Value"]))
    counters = sorted({c for d in names.values() for c in d})
    print("| kernel | dispatches | " + " | ".join(counters) + " |")
    print("|---|---:|" + "---:|" * len(counters))
    for k in sorted(names):
        d = names[k]
        nd = max(len(v) for v in d.values())
        cells = [f"{sum(d[c]) / len(d[c]):.4g}" if c in d else "" for c in counters]
        print(f"| {k} | {nd} | " + " | ".join(cells) + " |")


def _calibration(a):
    cf = counter_values(a.copy_fetch, "copy", "FETCH_SIZE")
    cw = counter_values(a.copy_write, "copy", "WRITE_SIZE")
    cf_mean = sum(sum(v) for v in cf.values()) / max(1, sum(len(v) for v in cf.values()))
    cw_mean = sum(sum(v) for v in cw.values()) / max(1, sum(len(v) for v in cw.values()))
    if cf_mean <= 0 or cw_mean <= 0:
        sys.exit("copy-kernel counters missing")
    return a.copy_bytes / (cf_mean * 1024.0), a.copy_bytes / (cw_mean * 1024.0)


def cmd_bandwidth(a):
    """Per kernel: trace duration and copy-calibrated HBM bytes per dispatch,
    hence the achieved HBM bandwidth against the peak."""
    kf, kw = _calibration(a)
    dur = {}
    for name, calls, avg, _tot in kernel_stats(a.trace, ""):
        dur[_short(name)] = (calls, avg)
    fv = counter_values(a.fetch, "", "FETCH_SIZE")
    wv = counter_values(a.write, "", "WRITE_SIZE")
    rows = []
    for name in fv:
        k = _short(name)
        if a.match and not any(m in k for m in a.match.split(",")):
            continue
        if k not in dur or name not in wv:
            continue
        rd = kf * 1024.0 * sum(fv[name]) / len(fv[name])
        wr = kw * 1024.0 * sum(wv[name]) / len(wv[name])
        calls, avg = dur[k]
        gbs = (rd + wr) / (avg * 1e-9) / 1e9
        rows.append((calls * avg, k, calls, avg, rd, wr, gbs))
    print(f"HBM peak {a.peak_gbs:.0f} GB/s; bytes per dispatch from FETCH_SIZE x {kf:.4f} "
          f"and WRITE_SIZE x {kw:.4f} KiB")
    print()
    print("| kernel | calls (trace) | avg us | read MB | written MB | GB/s | of peak |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for _t, k, calls, avg, rd, wr, gbs in sorted(rows, reverse=True):
        print(f"| {k} | {calls} | {avg / 1e3:.1f} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | "
              f"{gbs:.0f} | {gbs / a.peak_gbs:.2f} |")


def read_record(path):
    """The traffic record of a committed profile summary, or None."""
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("traffic-record:"):
                    return json.loads(line.split(":", 1)[1])
    except OSError:
        return None
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--match", default="k_filter<")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--match", default="k_filter<")
    t.add_argument("--workload", default="planted24k")
    t.add_argument("--last", type=int, default=0,
                   help="only each kernel's last N dispatches of the run (0: all)")
    t.add_argument("--kernel", default="", choices=[""] + sorted(KERNEL_SOURCES),
                   help="kernel whose sources the record's digest covers "
                        "(default: k_filter32 or k_filter, from --match)")
    bw = sub.add_parser("bandwidth")
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write"):
        bw.add_argument("--" + k.replace("_", "-"), required=True)
    bw.add_argument("--copy-bytes", type=float, required=True)
    bw.add_argument("--match", default="",
                    help="comma-separated substrings of the kernels to list (all if empty)")
    bw.add_argument("--peak-gbs", type=float, default=8000.0)
    tr = sub.add_parser("trace")
    tr.add_argument("dir")
    tr.add_argument("--match", default="k_filter<")
    tr.add_argument("--last", type=int, default=0,
                    help="only each kernel's last N dispatches of the run (0: all)")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--match", default="k_filter<")
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters,
     "bandwidth": cmd_bandwidth, "trace": cmd_trace}[a.cmd](a)


if __name__ == "__main__":
    main()
