"""Replay a timed query stream against a gp.Server and summarise latency.

The server (include/gp.h, gp_server_*) does the batching on the device; this
module only submits queries at their arrival times and collects outcomes.
"""
from __future__ import annotations

import time

import numpy as np


def run_stream(server, stream, patterns, time_scale: float = 1.0, note=None) -> list:
    """Submit each (t, graph, pattern) query at t * time_scale seconds after
    the start; wait for all; return one dict per query."""
    t0 = time.perf_counter()
    tickets = []
    for i, (t, g, p) in enumerate(stream):
        delay = t0 + t * time_scale - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        k, edges = patterns[p]
        tickets.append(server.submit(g, k, edges))
        if note and (i + 1) % 500 == 0:
            note(f"submitted {i + 1}/{len(stream)}")
    out = []
    last = time.perf_counter()
    for i, ((t, g, p), tk) in enumerate(zip(stream, tickets)):
        while True:
            try:
                st, c, lat = server.wait(tk, 5.0)
                break
            except RuntimeError as e:  # GP_ERR_TIMEOUT: still running; report progress
                if getattr(e, "status", None) != -13:
                    raise
                if note:
                    note(f"waiting: {i}/{len(stream)} collected, {server.stats()}")
        if note and time.perf_counter() - last > 10.0:
            last = time.perf_counter()
            note(f"collected {i + 1}/{len(stream)}")
        out.append({"graph": g, "pattern": p, "status": st, "count": c, "latency_s": lat})
    wall = time.perf_counter() - t0
    for r in out:
        r["wall_s"] = wall
    return out


def summarise(results: list) -> dict:
    ok = [r for r in results if r["status"] == 0]
    lat = np.array([r["latency_s"] for r in ok]) if ok else np.zeros(1)
    wall = results[0]["wall_s"] if results else 0.0
    return {
        "queries": len(results),
        "completed": len(ok),
        "rejected_budget": sum(r["status"] == -10 for r in results),
        "overflow": sum(r["status"] == -9 for r in results),
        "failed_other": sum(r["status"] not in (0, -9, -10) for r in results),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "qps": len(results) / wall if wall > 0 else 0.0,
        "wall_s": wall,
    }
