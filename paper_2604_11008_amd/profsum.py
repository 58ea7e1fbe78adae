"""Summaries of rocprofv3 CSV output, and the per-launch HBM traffic record
that bench.py reports.

Traffic of a kernel = FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two
separate `rocprofv3 --pmc` runs, each scaled by what the same counter reads
for a plain device copy of known size in the same run (bench.py always
runs a torch copy of 1 GiB, i.e. 1 GiB read and 1 GiB written).  The
record carries a hash of the kernel sources and of the workload generator;
once either changes, the record no longer applies and bench.py reports
traffic as null.

Usage (after the rocprofv3 runs):
  python -m paper_2604_11008_amd.profsum stats  <kernel_stats.csv>
  python -m paper_2604_11008_amd.profsum trace  <kernel_trace.csv> <kernel substring> <skip> <count>
  python -m paper_2604_11008_amd.profsum counters <counter_collection.csv>
  python -m paper_2604_11008_amd.profsum traffic <fetch.csv> <write.csv> <kernel substring> <out.json>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
# the kernel sources and the workload generator (the traffic depends on both)
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("pm_device.h", "pm_step_f64.hip",
                                                    "pm_step_f32.hip", "pm_mac_f64.hip",
                                                    "pm_mac_f32.hip", "pm_ilv_f64.hip",
                                                    "pm_ilv_f32.hip", "pm_staged_f64.hip",
                                                    "pm_staged_f32.hip", "pm_staged_ilv_f64.hip",
                                                    "pm_staged_ilv_f32.hip", "pm_kernels.hip",
                                                    "pm_internal.h")] + \
    [os.path.join(PKG, "gen.py")]
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


def source_hash(paths=SOURCES):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _get(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def stats(path, top=12):
    """Kernel name, calls, average and total duration (us) from kernel_stats.csv."""
    out = []
    for r in _rows(path)[:top]:
        name = _get(r, "Name", "KERNEL_NAME", "Kernel_Name")
        calls = int(_get(r, "Calls", "CALLS"))
        avg = float(_get(r, "AverageNs", "AVERAGE_NS")) / 1e3
        tot = float(_get(r, "TotalDurationNs", "TOTAL_DURATION_NS")) / 1e3
        out.append((name, calls, avg, tot))
    return out


def trace_window(path, substr, skip, count):
    """Durations (us) of the dispatches skip .. skip+count-1, in start order,
    of the kernels whose name contains substr (kernel_trace.csv)."""
    rows = [r for r in _rows(path) if substr in _get(r, "Kernel_Name", "KERNEL_NAME")]
    rows.sort(key=lambda r: int(_get(r, "Start_Timestamp", "START_TIMESTAMP")))
    d = [(int(_get(r, "End_Timestamp", "END_TIMESTAMP")) -
          int(_get(r, "Start_Timestamp", "START_TIMESTAMP"))) / 1e3 for r in rows]
    return d[skip:skip + count], len(d)


def counter_means(path):
    """{kernel name: {counter: (mean value, dispatches)}} from counter_collection.csv."""
    acc = defaultdict(lambda: defaultdict(list))
    for r in _rows(path):
        k = _get(r, "Kernel_Name", "KERNEL_NAME", "Kernel-Name")
        c = _get(r, "Counter_Name", "COUNTER_NAME")
        v = float(_get(r, "Counter_Value", "COUNTER_VALUE"))
        acc[k][c].append(v)
    return {k: {c: (sum(v) / len(v), len(v)) for c, v in d.items()} for k, d in acc.items()}


def _kernel_value(means, substr, counter, largest=False):
    vals = [(c[counter][0], k) for k, c in means.items() if substr in k and counter in c]
    if not vals:
        raise KeyError(f"no {counter} for kernels matching {substr!r}")
    return max(vals)[0] if largest else vals[0][0]


COPY_DISPATCHES = 13  # bench.py's copy probe: 3 warm-up copies and 10 timed ones


def copy_reading(path, counter):
    """The counter's reading (KiB) for the 1 GiB copy: the median over the
    run's last COPY_DISPATCHES device copies, which are bench.py's copy probe
    (run after every pool copy; the counter runs pass --no-cpu, so no host
    copy follows it)."""
    rows = [r for r in _rows(path)
            if COPY_KERNEL in _get(r, "Kernel_Name", "KERNEL_NAME", "Kernel-Name") and
            _get(r, "Counter_Name", "COUNTER_NAME") == counter]
    rows.sort(key=lambda r: int(_get(r, "Dispatch_Id", "DISPATCH_ID")))
    vals = sorted(float(_get(r, "Counter_Value", "COUNTER_VALUE"))
                  for r in rows[-COPY_DISPATCHES:])
    if not vals or vals[len(vals) // 2] <= 0:
        raise KeyError(f"no {counter} reading for the copy kernel")
    return vals[len(vals) // 2]


def traffic(fetch_csv, write_csv, kernel_substr):
    fm, wm = counter_means(fetch_csv), counter_means(write_csv)
    fetch_kib = _kernel_value(fm, kernel_substr, "FETCH_SIZE")
    write_kib = _kernel_value(wm, kernel_substr, "WRITE_SIZE")
    f_copy = copy_reading(fetch_csv, "FETCH_SIZE")
    w_copy = copy_reading(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (f_copy * 1024)
    w_scale = COPY_BYTES / (w_copy * 1024)
    total = fetch_kib * 1024 * f_scale + write_kib * 1024 * w_scale
    return {"kernel": kernel_substr, "fetch_kib": round(fetch_kib, 1),
            "write_kib": round(write_kib, 1), "copy_fetch_kib": round(f_copy, 1),
            "copy_write_kib": round(w_copy, 1), "fetch_scale": round(f_scale, 4),
            "write_scale": round(w_scale, 4), "bytes_per_launch": int(total),
            "source_hash": source_hash()}


def load_traffic(path):
    """bytes_per_launch from a traffic record, or None if missing or stale."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def main(argv):
    if argv[0] == "stats":
        for name, calls, avg, tot in stats(argv[1]):
            print(f"{avg:12.2f} us avg {calls:6d} calls {tot:12.1f} us total  {name[:100]}")
    elif argv[0] == "trace":
        d, n = trace_window(argv[1], argv[2], int(argv[3]), int(argv[4]))
        if not d:
            raise SystemExit(f"{argv[2]}: {n} dispatches, none from index {argv[3]} on")
        print(f"{argv[2]}: dispatches {argv[3]}..{int(argv[3]) + len(d) - 1} of {n}: "
              f"mean {sum(d) / len(d):.2f} us, min {min(d):.2f}, max {max(d):.2f}, "
              f"first {d[0]:.2f}, last {d[-1]:.2f}")
    elif argv[0] == "counters":
        for k, d in counter_means(argv[1]).items():
            for c, (v, n) in sorted(d.items()):
                print(f"{c:32s} {v:18.1f}  (n={n})  {k[:80]}")
    elif argv[0] == "traffic":
        rec = traffic(argv[1], argv[2], argv[3])
        with open(argv[4], "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
