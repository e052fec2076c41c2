"""Summaries of rocprofv3 output for the measurement records under profiles/.

kernel_stats(csv)      -> per-kernel call count and average duration from --kernel-trace --stats.
counter_summary(...)   -> HBM bytes per launch of one kernel from two --pmc passes (FETCH_SIZE, then
                          WRITE_SIZE, both in KiB per dispatch), each scaled by what the same counter
                          reads for a reference copy of known size in the same run.
flop_rates(...)        -> per kernel: FP64 and FP32 vector FLOPs and bf16 matrix-core FLOPs per dispatch
                          from one --pmc pass over SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64,
                          SQ_INSTS_VALU_{ADD,MUL,FMA}_F32 and SQ_INSTS_VALU_MFMA_MOPS_BF16, divided by the
                          kernel's average duration from a --kernel-trace --stats run.
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


# MI355X peaks (vendor figures): FP64 vector 78.6 TFLOP/s, FP32 vector 157.3, dense bf16 matrix 2500
PEAKS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16_mfma": 2500.0}


def flop_rates(counter_csv: str, stats_csv: str, min_calls: int = 1) -> list[dict]:
    """A vector instruction counts 64 lanes (FMA: 2 FLOPs per lane; inactive lanes included, so an
    upper bound); one bf16 MFMA MOP is 512 FLOPs."""
    per = {}
    for r in csv.DictReader(open(counter_csv)):
        key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Dispatch_ID", "")))
        per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    by_kernel = {}
    for (name, _), c in per.items():
        f64 = 64 * (c.get("SQ_INSTS_VALU_ADD_F64", 0) + c.get("SQ_INSTS_VALU_MUL_F64", 0) +
                    c.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * c.get("SQ_INSTS_VALU_FMA_F64", 0))
        f32 = 64 * (c.get("SQ_INSTS_VALU_ADD_F32", 0) + c.get("SQ_INSTS_VALU_MUL_F32", 0) +
                    2 * c.get("SQ_INSTS_VALU_FMA_F32", 0))
        mf = 512 * c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0)
        by_kernel.setdefault(name, []).append((f64, f32, mf))
    dur = {k["name"]: k["avg_ns"] for k in kernel_stats(stats_csv)}
    out = []
    for name, rows in by_kernel.items():
        if len(rows) < min_calls or name not in dur:
            continue
        f64, f32, mf = (statistics.mean(v[i] for v in rows) for i in range(3))
        t = dur[name] * 1e-9
        rec = dict(kernel=name, dispatches=len(rows), avg_us=round(dur[name] / 1e3, 2),
                   fp64_flop=round(f64), fp32_flop=round(f32), bf16_mfma_flop=round(mf),
                   fp64_tflops=round(f64 / t / 1e12, 3), fp32_tflops=round(f32 / t / 1e12, 3),
                   bf16_mfma_tflops=round(mf / t / 1e12, 3))
        rec["fp64_frac"] = round(rec["fp64_tflops"] / PEAKS_TFLOPS["fp64"], 4)
        rec["fp32_frac"] = round(rec["fp32_tflops"] / PEAKS_TFLOPS["fp32"], 4)
        rec["bf16_mfma_frac"] = round(rec["bf16_mfma_tflops"] / PEAKS_TFLOPS["bf16_mfma"], 5)
        out.append(rec)
    return out


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(json.dumps(kernel_stats(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""), indent=1))
    elif sys.argv[1] == "flops":
        print(json.dumps(flop_rates(sys.argv[2], sys.argv[3]), indent=1))
    elif sys.argv[1] == "counters":
        print(json.dumps(counter_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5])), indent=1))
