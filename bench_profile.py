#!/usr/bin/env python3
"""Summaries of rocprofv3 output for bench.py (text/JSON under profiles/).

  stats:   kernel trace (--kernel-trace --stats) of a bench.py run -> a Markdown
           table: rocprofv3's own per-kernel statistics over every dispatch, and
           the per-dispatch statistics of the last N dispatches of each kernel
           (the timed, autotuned launches; the autotuner's candidates come first).
  mfma:    one --pmc run counting MFMA operations (SQ_INSTS_VALU_MFMA_MOPS_F32 /
           _F64, 512 flops each) and a kernel trace of the same command ->
           issued MFMA flops per dispatch of each MFMA kernel over its average
           traced duration, against the dense MFMA peak of its precision.
  counters: several --pmc passes of one command -> per-kernel medians of every
           counter and derived ratios (MFMA busy fraction, wait shares, LDS bank
           conflicts, instructions per MFMA).
  traffic: two --pmc runs of the same command (FETCH_SIZE, then WRITE_SIZE) ->
           HBM bytes per launch of one kernel, each counter scaled by the reading
           of the same counter for a plain device copy of known size (the
           bench's --copy-calibration copy), plus the sha256 of the kernel
           source, so that bench.py drops the figure once the kernels change.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(ROOT, "paper_2607_19489_amd", "csrc", "afmm_kernels.hip")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()


def short(name: str) -> str:
    name = re.sub(r"^void ", "", name)
    name = re.sub(r"\(.*$", "", name)
    return name.replace("afmm::", "")


def _find(d: str, suffix: str):
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        sys.exit(f"no *{suffix} under {d}")
    return hits[0]


def cmd_stats(a):
    stats = list(csv.DictReader(open(_find(a.trace, "kernel_stats.csv"))))
    trace = list(csv.DictReader(open(_find(a.trace, "kernel_trace.csv"))))
    per = {}
    for r in trace:
        k = short(r["Kernel_Name"])
        per.setdefault(k, []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = [f"# rocprofv3 kernel statistics: {a.title}", "", "Command (repository root on the MI355X box):", "",
           "```", a.command, "```", "",
           "## All dispatches (rocprofv3 --stats)", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:a.top]:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    out += ["", f"## Last {a.last} dispatches of each kernel (the timed launches after autotuning)", "",
            "| kernel | dispatches | avg us | median us | min us | max us |", "|---|---|---|---|---|---|"]
    rows = []
    for k, v in per.items():
        v.sort()
        d = [x[1] / 1e3 for x in v[-a.last:]]
        rows.append((sum(d), k, d))
    for tot, k, d in sorted(rows, reverse=True)[:a.top]:
        out.append(f"| `{k}` | {len(d)} | {statistics.mean(d):.1f} | {statistics.median(d):.1f} | "
                   f"{min(d):.1f} | {max(d):.1f} |")
    open(a.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def _pmc(d: str, counter: str):
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = (short(r["Kernel_Name"]), r.get("Dispatch_Id", ""))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    byk = {}
    for (k, did), v in per.items():
        byk.setdefault(k, []).append((int(did) if did.isdigit() else 0, v))
    for v in byk.values():
        v.sort()
    return byk


PEAK_TFLOPS = {"SQ_INSTS_VALU_MFMA_MOPS_F32": 157.3, "SQ_INSTS_VALU_MFMA_MOPS_F64": 78.6}


def cmd_mfma(a):
    trace = list(csv.DictReader(open(_find(a.trace, "kernel_trace.csv"))))
    dur = {}
    for r in trace:
        key = (short(r["Kernel_Name"]), r.get("Grid_Size_X") or r.get("Grid_Size"))
        dur.setdefault(key, []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows = list(csv.DictReader(open(_find(a.pmc, "counter_collection.csv"))))
    out = [f"# Issued MFMA throughput: {a.title}", "",
           "Operation counts (rocprofv3 --pmc, SQ_INSTS_VALU_MFMA_MOPS_*: multiply and add operations / 512,",
           "summed over the shader engines) per dispatch, over the median duration of the dispatches of the",
           "same kernel and grid in a kernel trace of the same command (last N of each).  Issued operations",
           "include the zero padding of the MFMA tiles; the useful-flop rate is the bench's own figure.  Every",
           "launch of a solve runs on the caller's one stream, so a traced duration is one launch alone.  The",
           "grids other than the autotuned one are the tuner's candidate tap splits.", "",
           "Commands (repository root on the MI355X box):", "", "```", a.command_pmc, a.command_trace, "```", "",
           "| kernel | grid | counter | dispatches | issued GFLOP / dispatch | median us (trace) | issued TFLOP/s | of peak |",
           "|---|---|---|---|---|---|---|---|"]
    for counter, peak in PEAK_TFLOPS.items():
        per = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            key = (short(r["Kernel_Name"]), r["Grid_Size"], r.get("Dispatch_Id", ""))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        byk = {}
        for (k, g, did), v in per.items():
            byk.setdefault((k, g), []).append((int(did) if did.isdigit() else 0, v))
        for (k, g), v in sorted(byk.items()):
            v.sort()
            ops = [x for _, x in v[-a.last:]]
            if not ops or max(ops) == 0 or (k, g) not in dur:
                continue
            d = sorted(dur[(k, g)])[-a.last:]
            us = statistics.median(x[1] for x in d) / 1e3
            gf = statistics.median(ops) * 512 / 1e9
            tf = gf / us * 1e3
            out.append(f"| `{k}` | {g} | {counter[-3:]} | {len(ops)} | {gf:.2f} | {us:.1f} | {tf:.1f} | {tf / peak:.1%} |")
    open(a.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def cmd_traffic(a):
    fetch = _pmc(a.fetch, "FETCH_SIZE")
    write = _pmc(a.write, "WRITE_SIZE")
    copy_bytes = a.copy_mib * 1024 * 1024
    cf = max(v for _, v in fetch[COPY_KERNEL])   # KiB per dispatch of the calibration copy
    cw = max(v for _, v in write[COPY_KERNEL])
    f_factor = copy_bytes / (cf * 1024.0)
    w_factor = copy_bytes / (cw * 1024.0)
    k = a.kernel
    fk = [v for _, v in fetch[k][-a.last:]]
    wk = [v for _, v in write[k][-a.last:]]
    fb = statistics.median(fk) * 1024.0 * f_factor
    wb = statistics.median(wk) * 1024.0 * w_factor
    res = {"kernel": k, "workload": a.workload, "source_sha256": source_hash(), "command_fetch": a.command_fetch,
           "command_write": a.command_write, "dispatches_used": len(fk),
           "fetch_kib_per_dispatch": statistics.median(fk), "write_kib_per_dispatch": statistics.median(wk),
           "calibration": {"copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
                           "fetch_factor": f_factor, "write_factor": w_factor},
           "traffic_bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb}
    json.dump(res, open(a.out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def cmd_counters(a):
    """Counter passes (--pmc runs of one command, one directory each) -> per-kernel
    medians over the last N dispatches, with the durations of a kernel trace of
    the same command; plus ratios that say where the waves' time goes."""
    vals = {}
    for d in a.pmc:
        for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
            k = short(r["Kernel_Name"])
            if a.kernels and k not in a.kernels:
                continue
            key = (k, r["Counter_Name"], r.get("Dispatch_Id", ""))
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    per = {}
    for (k, c, did), v in vals.items():
        per.setdefault((k, c), []).append((int(did) if did.isdigit() else 0, v))
    med = {}
    for (k, c), v in per.items():
        v.sort()
        med[(k, c)] = statistics.median(x for _, x in v[-a.last:])
    dur = {}
    if a.trace:
        for r in csv.DictReader(open(_find(a.trace, "kernel_trace.csv"))):
            k = short(r["Kernel_Name"])
            dur.setdefault(k, []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    kernels = a.kernels or sorted({k for k, _ in med})
    counters = sorted({c for _, c in med})
    out = [f"# Hardware counters: {a.title}", "",
           "Median over the last dispatches of each kernel (the timed launches) of each counter, summed over",
           "the GPU's shader engines / instances, one rocprofv3 --pmc pass per group of counters (no pass",
           "exceeds the hardware's counter slots).  Cycle counters named *_CYCLES are per SIMD or per wave as",
           "rocprofv3 documents them; SQ_WAVE_CYCLES, SQ_WAIT_* and SQ_BUSY_CU_CYCLES are in quad-cycles.", "",
           "Commands (repository root on the MI355X box):", "", "```", *a.command, "```", "",
           "| counter | " + " | ".join(f"`{k}`" for k in kernels) + " |", "|---|" + "---|" * len(kernels)]
    for c in counters:
        out.append(f"| {c} | " + " | ".join(f"{med[(k, c)]:.4g}" if (k, c) in med else "" for k in kernels) + " |")
    out += ["", "## Derived", ""]
    rows = []

    def g(k, c):
        return med.get((k, c))
    for k in kernels:
        r = {"kernel": k}
        if k in dur:
            d = sorted(dur[k])[-a.last:]
            r["us"] = statistics.median(x[1] for x in d) / 1e3
        cyc = r.get("us", 0) * 1e-6 * a.clock_ghz * 1e9
        if g(k, "SQ_VALU_MFMA_BUSY_CYCLES") and cyc:
            r["mfma_busy"] = g(k, "SQ_VALU_MFMA_BUSY_CYCLES") / (cyc * a.simds)
        wc = g(k, "SQ_WAVE_CYCLES")
        if wc:
            for c in ("SQ_WAIT_INST_ANY", "SQ_WAIT_ANY", "SQ_ACTIVE_INST_ANY", "SQ_WAIT_INST_LDS"):
                if g(k, c) is not None:
                    r[c[3:].lower() + "/wave_cycles"] = g(k, c) / wc
            if cyc:
                r["wave_occupancy_index"] = 4.0 * wc / (cyc * a.simds)
        if g(k, "TA_TA_BUSY_sum") is not None and cyc:
            r["ta_busy"] = g(k, "TA_TA_BUSY_sum") / (cyc * a.cus)
            if g(k, "TA_ADDR_STALLED_BY_TC_CYCLES_sum") is not None and g(k, "TA_TA_BUSY_sum"):
                r["ta_addr_stalled_by_tcp/ta_busy"] = g(k, "TA_ADDR_STALLED_BY_TC_CYCLES_sum") / g(k, "TA_TA_BUSY_sum")
        if g(k, "TCP_PENDING_STALL_CYCLES_sum") is not None and cyc:
            r["tcp_pending_stall"] = g(k, "TCP_PENDING_STALL_CYCLES_sum") / (cyc * a.cus)
        if g(k, "TCP_READ_TAGCONFLICT_STALL_CYCLES_sum") is not None and cyc:
            r["tcp_tagconflict_stall"] = g(k, "TCP_READ_TAGCONFLICT_STALL_CYCLES_sum") / (cyc * a.cus)
        if g(k, "TCP_TCC_READ_REQ_LATENCY_sum") is not None and g(k, "TCP_TCC_READ_REQ_sum"):
            r["l2_read_latency_cycles"] = g(k, "TCP_TCC_READ_REQ_LATENCY_sum") / g(k, "TCP_TCC_READ_REQ_sum")
        if g(k, "SQ_LDS_BANK_CONFLICT") is not None and g(k, "SQ_ACTIVE_INST_LDS"):
            r["lds_bank_conflict/active_lds"] = g(k, "SQ_LDS_BANK_CONFLICT") / g(k, "SQ_ACTIVE_INST_LDS")
        mf = g(k, "SQ_INSTS_MFMA") or g(k, "SQ_INSTS_VALU_MFMA_F32")
        if mf:
            for c in ("SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_SALU", "SQ_INSTS_VALU"):
                if g(k, c) is not None:
                    r[c[9:].lower() + "/mfma"] = g(k, c) / mf
        rows.append(r)
    keys = []
    for r in rows:
        keys += [x for x in r if x not in keys and x != "kernel"]
    out.append("| kernel | " + " | ".join(keys) + " |")
    out.append("|---|" + "---|" * len(keys))
    for r in rows:
        out.append(f"| `{r['kernel']}` | " + " | ".join(f"{r[x]:.3g}" if x in r else "" for x in keys) + " |")
    open(a.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--last", type=int, default=20)
    s.add_argument("--top", type=int, default=14)
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("--pmc", required=True)
    m.add_argument("--trace", required=True)
    m.add_argument("--last", type=int, default=8)
    m.add_argument("--title", required=True)
    m.add_argument("--command-pmc", required=True)
    m.add_argument("--command-trace", required=True)
    m.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--last", type=int, default=20)
    t.add_argument("--copy-mib", type=int, default=256)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--pmc", required=True, nargs="+")
    c.add_argument("--trace")
    c.add_argument("--kernels", nargs="*")
    c.add_argument("--last", type=int, default=5)
    c.add_argument("--clock-ghz", type=float, default=2.4)
    c.add_argument("--simds", type=int, default=1024)
    c.add_argument("--cus", type=int, default=256)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True, nargs="+")
    c.add_argument("--out", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "mfma": cmd_mfma, "traffic": cmd_traffic, "counters": cmd_counters}[a.mode](a)


if __name__ == "__main__":
    main()
