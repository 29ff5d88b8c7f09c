"""Summaries of rocprofv3 output for the measurements bench.py reports.

HBM traffic of a kernel comes from two counter runs (FETCH_SIZE, then
WRITE_SIZE, each in KiB per dispatch). Each counter is scaled by what it
reads for a plain device copy of known size in the same run (a 1 GiB copy
reads and writes 1 GiB), which calibrates the counter's unit and coverage.
A summary records a hash of the kernel sources; it stops applying as soon
as they change.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/count_kernel.hpp", "csrc/sets.hpp", "csrc/count_inst.hip", "csrc/count.hip",
                  "csrc/count_batch.hip", "csrc/plan_desc.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(path: str):
    """The traffic summary at path, if it matches the current kernel sources."""
    try:
        with open(path) as f:
            tr = json.load(f)
    except (OSError, ValueError):
        return None
    return tr if tr.get("kernel_source_hash") == kernel_source_hash() else None


def _rows(path_glob: str):
    for path in sorted(glob.glob(path_glob, recursive=True)):
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def _db_rows(path_glob: str, counter: str):
    """(dispatch id, kernel name, value) rows of one counter from rocprofv3's
    SQLite output (its counters_collection view)."""
    import sqlite3
    for path in sorted(glob.glob(path_glob, recursive=True)):
        con = sqlite3.connect(f"file:{path}?mode=ro", uri=True)
        try:
            yield from con.execute("SELECT dispatch_id, kernel_name, value FROM counters_collection "
                                   "WHERE counter_name = ?", (counter,))
        finally:
            con.close()


def counter_per_dispatch(path_glob: str, counter: str) -> list:
    """[(dispatch id, kernel name, value)] for one counter from rocprofv3
    counter_collection CSV files or its SQLite databases (*.db), values
    summed over the counter's instances."""
    acc: dict = {}
    if path_glob.endswith(".db"):
        for did, kern, val in _db_rows(path_glob, counter):
            key = (int(did), kern)
            acc[key] = acc.get(key, 0.0) + float(val)
        return [(d, k, v) for (d, k), v in sorted(acc.items())]
    for r in _rows(path_glob):
        name = r.get("Counter_Name") or r.get("counter_name")
        if name != counter:
            continue
        did = int(r.get("Dispatch_Id") or r.get("dispatch_id") or 0)
        kern = r.get("Kernel_Name") or r.get("kernel_name") or ""
        val = float(r.get("Counter_Value") or r.get("counter_value") or 0.0)
        key = (did, kern)
        acc[key] = acc.get(key, 0.0) + val
    return [(d, k, v) for (d, k), v in sorted(acc.items())]


def traffic_summary(fetch_glob: str, write_glob: str, kernel_match: str, copy_bytes: int,
                    pattern: str, workload: str, plan: dict | None = None,
                    l2_glob: str | None = None) -> dict:
    """HBM bytes of the longest dispatch whose name contains kernel_match,
    with FETCH_SIZE / WRITE_SIZE scaled by the copy kernel's readings; plus
    the L2 hit rate (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)) if given.
    `plan` records the configuration the counters were taken with."""
    fetch = counter_per_dispatch(fetch_glob, "FETCH_SIZE")
    write = counter_per_dispatch(write_glob, "WRITE_SIZE")

    def copy_value(rows):
        vals = [v for _, k, v in rows if "copyBuffer" in k or "copy" in k.lower()]
        return max(vals) if vals else None

    def kernel_value(rows):
        vals = [v for _, k, v in rows if kernel_match in k]
        return max(vals) if vals else None

    cf, cw = copy_value(fetch), copy_value(write)
    kf, kw = kernel_value(fetch), kernel_value(write)
    # counters read KiB; the copy moves copy_bytes each way
    f_scale = copy_bytes / (cf * 1024.0) if cf else None
    w_scale = copy_bytes / (cw * 1024.0) if cw else None
    hbm = None
    if None not in (f_scale, w_scale, kf, kw):
        hbm = kf * 1024.0 * f_scale + kw * 1024.0 * w_scale
    l2 = None
    if l2_glob:
        hit = kernel_value(counter_per_dispatch(l2_glob, "TCC_HIT_sum"))
        miss = kernel_value(counter_per_dispatch(l2_glob, "TCC_MISS_sum"))
        if hit is not None and miss is not None and hit + miss > 0:
            l2 = {"hits": hit, "misses": miss, "hit_rate": hit / (hit + miss)}
    return {"workload": workload, "pattern": pattern, "kernel_match": kernel_match,
            "fetch_kib": kf, "write_kib": kw, "copy_fetch_kib": cf, "copy_write_kib": cw,
            "copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
            "hbm_bytes_per_launch": hbm, "l2": l2, "plan": plan,
            "kernel_source_hash": kernel_source_hash()}


def same_plan(a: dict | None, b: dict | None) -> bool:
    """Whether two recorded configurations (order, restrictions, launch, and
    whether the last two levels are counted with inclusion-exclusion) agree."""
    if not a or not b:
        return False
    keys = ("order", "restrictions", "launch")
    return (all(json.dumps(a.get(k), sort_keys=True) == json.dumps(b.get(k), sort_keys=True) for k in keys)
            and bool(a.get("iep", False)) == bool(b.get("iep", False)))


def main(argv):
    """python -m paper_2009_10955_amd.profiling FETCH_GLOB WRITE_GLOB KERNEL_MATCH COPY_MIB
    PATTERN WORKLOAD OUT [--plans BENCH_JSON] [--l2 L2_GLOB]"""
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_2009_10955_amd.profiling")
    for name in ("fetch_glob", "write_glob", "kernel_match", "copy_mib", "pattern", "workload", "out"):
        ap.add_argument(name)
    ap.add_argument("--plans", help="bench.py output whose plan for PATTERN the counters ran")
    ap.add_argument("--l2", help="counter files with TCC_HIT_sum and TCC_MISS_sum")
    a = ap.parse_args(argv)
    plan = None
    if a.plans:
        with open(a.plans) as f:
            plans = json.loads(f.read().strip().splitlines()[-1])["plans"]

        def pick(p):
            return {k: p[k] for k in ("order", "restrictions", "launch")} | {"iep": bool(p.get("iep", False))}
        # PATTERN "all": a batched launch of every plan of the run
        plan = {n: pick(p) for n, p in plans.items()} if a.pattern == "all" else pick(plans[a.pattern])
    s = traffic_summary(a.fetch_glob, a.write_glob, a.kernel_match, int(a.copy_mib) << 20, a.pattern,
                        a.workload, plan, a.l2)
    with open(a.out, "w") as f:
        json.dump(s, f, indent=1)
    print(json.dumps(s))


if __name__ == "__main__":
    main(sys.argv[1:])
