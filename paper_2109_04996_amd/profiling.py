"""Summaries of rocprofv3 output for the measurement records under profiles/.

kernel_stats(csv)      -> per-kernel call count and average duration from --kernel-trace --stats.
counter_summary(...)   -> HBM bytes per launch of one kernel from two --pmc passes (FETCH_SIZE, then
                          WRITE_SIZE, both in KiB per dispatch), each scaled by what the same counter
                          reads for a reference copy of known size in the same run.
"""
from __future__ import annotations

import csv
import json
import statistics
import sys


def kernel_stats(path: str, match: str = "") -> list[dict]:
    out = []
    for r in csv.DictReader(open(path)):
        if match in r["Name"]:
            out.append(dict(name=r["Name"], calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                            min_ns=float(r["MinNs"]), max_ns=float(r["MaxNs"]), percent=float(r["Percentage"])))
    return out


def _per_dispatch(path: str, counter: str):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows]


def counter_summary(fetch_csv: str, write_csv: str, kernel_match: str, copy_bytes: int,
                    copy_match: str = "copyBuffer") -> dict:
    """Scale factors come from the largest copy dispatch (the reference copy of copy_bytes bytes)."""
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")
    half = copy_bytes // 2  # bytes read = bytes written
    cf = max((v for k, g, v in f if copy_match in k), default=None)
    cw = max((v for k, g, v in w if copy_match in k), default=None)
    fk = [v for k, g, v in f if kernel_match in k]
    wk = [v for k, g, v in w if kernel_match in k]
    fetch_factor = half / (cf * 1024.0)
    write_factor = half / (cw * 1024.0)
    fetch = statistics.mean(fk) * 1024.0 * fetch_factor
    write = statistics.mean(wk) * 1024.0 * write_factor
    return dict(kernel=kernel_match, launches=len(fk), fetch_kib_raw=statistics.mean(fk),
                write_kib_raw=statistics.mean(wk), copy_fetch_kib=cf, copy_write_kib=cw,
                fetch_factor=round(fetch_factor, 4), write_factor=round(write_factor, 4),
                fetch_bytes_per_launch=round(fetch), write_bytes_per_launch=round(write),
                hbm_bytes_per_launch=round(fetch + write))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(json.dumps(kernel_stats(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""), indent=1))
    elif sys.argv[1] == "counters":
        print(json.dumps(counter_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5])), indent=1))
