"""Summaries of rocprofv3 output for the profiles this repository keeps.

rocprofv3 writes one CSV row per (kernel dispatch, counter) with
``--pmc`` and one row per dispatch with ``--kernel-trace``.  These helpers
read those files and average a kernel's counters over a chosen range of its
dispatches (for example the launches of the steps a benchmark line timed),
so that a committed summary states exactly which launches it covers.
Plain CSV parsing; no GPU.
"""
from __future__ import annotations

import csv
from collections import OrderedDict
from typing import Dict, List, Optional


def read_counters(path: str) -> List[dict]:
    """Dispatches of a ``--pmc`` counter_collection.csv in dispatch order:
    {"dispatch", "kernel", "grid", "block", "lds", "vgpr", "counters": {name: value}}."""
    out: "OrderedDict[int, dict]" = OrderedDict()
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            rec = out.get(d)
            if rec is None:
                rec = {"dispatch": d, "kernel": row["Kernel_Name"], "grid": int(row["Grid_Size"]),
                       "block": int(row["Workgroup_Size"]), "lds": int(row["LDS_Block_Size"]),
                       "vgpr": int(row["VGPR_Count"]), "counters": {}}
                out[d] = rec
            rec["counters"][row["Counter_Name"]] = rec["counters"].get(row["Counter_Name"], 0.0) + float(
                row["Counter_Value"])
    return list(out.values())


def read_trace(path: str) -> List[dict]:
    """Dispatches of a ``--kernel-trace`` kernel_trace.csv: kernel name and
    duration in microseconds, in dispatch order."""
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out.append({"dispatch": int(row["Dispatch_Id"]), "kernel": row["Kernel_Name"],
                        "us": (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3})
    out.sort(key=lambda r: r["dispatch"])
    return out


def select(recs: List[dict], kernel: str, last: Optional[int] = None, first: int = 0) -> List[dict]:
    """Dispatches whose kernel name contains `kernel`; of those, the range
    [first, first + last) counted from the end when `last` is given
    (``last=20`` = the final 20 launches), else all from `first`."""
    sel = [r for r in recs if kernel in r["kernel"]]
    if last is not None:
        sel = sel[len(sel) - last - first: len(sel) - first]
    else:
        sel = sel[first:]
    return sel


def mean_counters(recs: List[dict]) -> Dict[str, float]:
    """Per-dispatch mean of every counter over `recs`."""
    if not recs:
        return {}
    keys = set().union(*[r["counters"].keys() for r in recs])
    return {k: sum(r["counters"].get(k, 0.0) for r in recs) / len(recs) for k in sorted(keys)}


def kernel_table(trace: List[dict]) -> List[dict]:
    """Per kernel: calls, average / min / max microseconds, total ms and share,
    largest total first (the --stats view of a trace)."""
    by: "OrderedDict[str, List[float]]" = OrderedDict()
    for r in trace:
        by.setdefault(r["kernel"], []).append(r["us"])
    tot = sum(sum(v) for v in by.values()) or 1.0
    rows = [{"kernel": k, "calls": len(v), "avg_us": sum(v) / len(v), "min_us": min(v), "max_us": max(v),
             "total_ms": sum(v) * 1e-3, "pct": 100.0 * sum(v) / tot} for k, v in by.items()]
    rows.sort(key=lambda r: -r["total_ms"])
    return rows


def copy_scale(recs: List[dict], counter: str, bytes_copied: int) -> Optional[float]:
    """Bytes per counter unit from the plain device copy of known size that
    ``bench.py --calib-copy`` runs first: the largest copy dispatch of the
    run (FETCH_SIZE and WRITE_SIZE count KiB)."""
    cands = [r for r in recs if "copy" in r["kernel"].lower() and counter in r["counters"]]
    if not cands:
        return None
    r = max(cands, key=lambda x: x["counters"][counter])
    v = r["counters"][counter]
    return bytes_copied / (v * 1024.0) if v > 0 else None


LDS_COUNTERS = ("SQ_INSTS_LDS_ATOMIC", "SQ_INSTS_LDS_LOAD", "SQ_INSTS_LDS_STORE", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH",
                "SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH", "SQ_LDS_ADDR_CONFLICT",
                "SQ_LDS_DATA_FIFO_FULL")


def window_record(fetch_csv: str, write_csv: str, sq_csv: Optional[str], launches: int,
                  copy_bytes: int = 512 << 20, lds_csv: Optional[str] = None) -> dict:
    """Counter figures of the particle kernel over its last `launches`
    dispatches (the benchmark's replayed window): HBM bytes per launch from
    FETCH_SIZE and WRITE_SIZE scaled by the calibration copy, the SQ
    instruction counts per launch when an SQ pass is given, and the LDS
    instruction mix (loads, stores, atomics and their bandwidth counters)
    when an LDS pass is given."""
    F, W = read_counters(fetch_csv), read_counters(write_csv)
    fs, ws = copy_scale(F, "FETCH_SIZE", copy_bytes), copy_scale(W, "WRITE_SIZE", copy_bytes)
    mf = mean_counters(select(F, "push_kernel", last=launches))
    mw = mean_counters(select(W, "push_kernel", last=launches))
    rec = {"launches": launches, "fetch_kib": mf.get("FETCH_SIZE"), "write_kib": mw.get("WRITE_SIZE"),
           "fetch_scale": fs, "write_scale": ws}
    if fs and ws and rec["fetch_kib"] is not None and rec["write_kib"] is not None:
        rec["bytes_per_launch"] = rec["fetch_kib"] * 1024.0 * fs + rec["write_kib"] * 1024.0 * ws
    if sq_csv:
        ms = mean_counters(select(read_counters(sq_csv), "push_kernel", last=launches))
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_WAVES", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS",
                  "SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES", "SQ_LDS_IDX_ACTIVE"):
            if k in ms:
                rec[k] = ms[k]
        if "SQ_INSTS_VALU" in ms:
            rec["valu_insts_per_launch"] = ms["SQ_INSTS_VALU"]
    if lds_csv:
        ml = mean_counters(select(read_counters(lds_csv), "push_kernel", last=launches))
        for k in LDS_COUNTERS:
            if k in ml:
                rec[k] = ml[k]
    return rec


def counter_table(csv_path: str, kernel: str, last: int) -> List[tuple]:
    """(counter, per-dispatch mean) of `kernel`'s last `last` dispatches."""
    return sorted(mean_counters(select(read_counters(csv_path), kernel, last=last)).items())


def _main(argv=None):
    import argparse
    import json
    import os
    import sys
    ap = argparse.ArgumentParser(description="summaries of rocprofv3 output for profiles/")
    sub = ap.add_subparsers(dest="cmd", required=True)
    w = sub.add_parser("window", help="particle-kernel counters of a step window -> traffic.json")
    w.add_argument("--workload", required=True)
    w.add_argument("--first", type=int, required=True)
    w.add_argument("--last", type=int, required=True)
    w.add_argument("--fetch", required=True)
    w.add_argument("--write", required=True)
    w.add_argument("--sq")
    w.add_argument("--lds")
    w.add_argument("--out", required=True)
    w.add_argument("--command", default="")
    t = sub.add_parser("trace", help="kernel table of a --kernel-trace run (markdown)")
    t.add_argument("csv")
    c = sub.add_parser("counters", help="mean counters of one kernel's last launches (markdown)")
    c.add_argument("csv")
    c.add_argument("--kernel", required=True)
    c.add_argument("--last", type=int, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        print(f"| counter | mean per launch ({a.kernel}, last {a.last}) |\n|---|---|")
        for k, v in counter_table(a.csv, a.kernel, a.last):
            print(f"| {k} | {v:.6g} |")
        return 0
    if a.cmd == "trace":
        print("| kernel | calls | avg µs | min µs | max µs | total ms | % |\n|---|---|---|---|---|---|---|")
        for r in kernel_table(read_trace(a.csv)):
            name = r["kernel"].split("(")[0].replace("void ", "")
            print(f"| `{name}` | {r['calls']} | {r['avg_us']:.1f} | {r['min_us']:.1f} | {r['max_us']:.1f} | "
                  f"{r['total_ms']:.2f} | {r['pct']:.1f} |")
        return 0
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, here)
    import bench
    rec = window_record(a.fetch, a.write, a.sq, a.last - a.first, lds_csv=a.lds)
    rec["command"] = a.command
    data = json.load(open(a.out)) if os.path.exists(a.out) else {}
    pk = data.setdefault("push_kernel", {})
    sha = bench.kernel_source_hash()
    if pk.get("workload") != a.workload or pk.get("source_sha") != sha:
        pk.clear()
    pk["workload"] = a.workload
    pk["source_sha"] = sha
    pk["source_sha_note"] = ("sha256 of k_push.hip, part.h, sdmd_dev.h with comments and whitespace removed "
                             "(bench.kernel_source_hash)")
    pk.setdefault("windows", {})[f"{a.first}-{a.last}"] = rec
    with open(a.out, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps(rec, indent=1))
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
