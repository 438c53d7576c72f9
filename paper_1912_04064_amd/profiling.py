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
