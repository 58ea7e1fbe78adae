"""The rocprofv3 summaries behind the committed profiles and the benchmark's
`traffic` figure: timed windows taken in start order, the per-launch bytes
scaled by the same counter's reading for the 1 GiB copy at the end of the
run (its last 13 copy dispatches; earlier, larger copies ignored), and a
traffic record that applies only while the kernel sources are unchanged."""
import csv
import json

import pytest

from paper_2604_11008_amd import profsum

KERNEL = "k_step<256, 4, double, false, false, 0>"
COPY = profsum.COPY_KERNEL


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)
    return str(path)


def _counters(path, counter, kernel_values, copy_values, big_copy=None):
    """One row per dispatch: the kernel's dispatches, then (optionally) eight
    large pool copies, then the copy probe's dispatches; the rows are written
    in reverse dispatch order."""
    rows, d = [], 0
    for v in kernel_values:
        d += 1
        rows.append([d, KERNEL, counter, v])
    for _ in range(8 if big_copy is not None else 0):
        d += 1
        rows.append([d, COPY, counter, big_copy])
    for v in copy_values:
        d += 1
        rows.append([d, COPY, counter, v])
    return _write(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
                  rows[::-1])


def test_trace_window_is_in_start_order(tmp_path):
    # dispatches listed out of order; durations 1, 2, ..., 6 us by start time
    rows = []
    for i in (3, 0, 5, 1, 4, 2):
        start = 1_000_000 * (i + 1)
        rows.append([KERNEL, start, start + 1000 * (i + 1)])
    rows.append(["other_kernel", 10, 20])
    p = _write(tmp_path / "t.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    d, n = profsum.trace_window(p, "k_step<", 2, 3)
    assert n == 6
    assert d == [3.0, 4.0, 5.0]


def test_stats_reads_microseconds(tmp_path):
    p = _write(tmp_path / "s.csv", ["Name", "Calls", "AverageNs", "TotalDurationNs"],
               [[KERNEL, 4, 2500.0, 10000.0]])
    assert profsum.stats(p) == [(KERNEL, 4, 2.5, 10.0)]


def test_traffic_scales_each_counter_by_the_copy(tmp_path, monkeypatch):
    n_copy = profsum.COPY_DISPATCHES
    # the copy of 1 GiB reads as half its size on FETCH_SIZE (factor 2) and as
    # its size on WRITE_SIZE (factor 1); one outlier among the probe's
    # dispatches and the larger copies before it do not move the median
    fetch_copy = [524288.0] * (n_copy - 1) + [600000.0]
    write_copy = [1048576.0] * n_copy
    f = _counters(tmp_path / "f.csv", "FETCH_SIZE", [1000.0, 3000.0], fetch_copy,
                  big_copy=5e6)
    w = _counters(tmp_path / "w.csv", "WRITE_SIZE", [500.0, 700.0], write_copy,
                  big_copy=9e6)
    rec = profsum.traffic(f, w, KERNEL)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_kib"] == 2000.0 and rec["write_kib"] == 600.0
    assert rec["bytes_per_launch"] == 2000 * 1024 * 2 + 600 * 1024
    assert rec["source_hash"] == profsum.source_hash()
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    assert profsum.load_traffic(str(path)) == rec["bytes_per_launch"]
    # a record of other kernel sources no longer applies
    monkeypatch.setattr(profsum, "source_hash", lambda paths=None: "0" * 16)
    assert profsum.load_traffic(str(path)) is None
    assert profsum.load_traffic(str(tmp_path / "missing.json")) is None


def test_traffic_without_a_copy_reading_is_an_error(tmp_path):
    f = _counters(tmp_path / "f.csv", "FETCH_SIZE", [1000.0], [])
    w = _counters(tmp_path / "w.csv", "WRITE_SIZE", [500.0], [])
    with pytest.raises(KeyError):
        profsum.traffic(f, w, KERNEL)

