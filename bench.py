#!/usr/bin/env python3
"""Benchmark of the exact embedding-counting path on one MI355X.

Workload (default): R-MAT scale 22 (4,194,304 vertices, edge factor 8,
a=0.57 b=0.19 c=0.19 d=0.05, seed 4; symmetrised, no self-loops or
duplicates) with the patterns 4-clique, house, 5-cycle and 6-cycle+chord.
Every pattern is planned, estimated and tuned first; those whose tuned full
run is estimated within --max-pattern-s are timed. A step counts one of 20
strided slices of every timed pattern's root edges with the batched launches
(one hipGraph), and the same slices are counted again with one launch per
pattern; 20 steps count every embedding once. Inputs (graph layout, plans)
are resident before timing starts, as the paper times only the matching
(graph loading and preprocessing excluded).

Prints ONE JSON line: embeddings/s over the timed steps, the batched
launch's algorithmic bytes per second against the HBM roofline, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "embeddings/s + intersection HBM GB/s; batched-vs-plain speedup, exact counts"

WORKLOADS = {
    # name: (config graph index, patterns, description, mode)
    "rmat17": (1, ["house", "5-cycle", "5-clique"],
               "R-MAT scale 17, edge factor 8, (0.57,0.19,0.19,0.05), seed 2; house, 5-cycle, "
               "5-clique, one launch each", "plain"),
    "er1000": (0, ["triangle", "4-cycle", "4-clique"],
               "G(1000, 0.01) seed 1; triangle, 4-cycle, 4-clique, one launch each", "plain"),
    "chunglu7000": (2, ["6-cycle", "6-cycle-chord", "prism", "k4-path", "5-wheel", "6-clique"],
                    "Chung-Lu n=7000, gamma 2.1, ~100k edges, seed 3; six 6-vertex patterns counted "
                    "by one batched hipGraph replay, against one launch per pattern",
                    "batched"),
    "rmat22": (3, ["4-clique", "house", "5-cycle", "6-cycle-chord"],
               "R-MAT scale 22, edge factor 8, (0.57,0.19,0.19,0.05), seed 4; 4-clique, house, "
               "5-cycle, 6-cycle+chord counted by one batched hipGraph replay against one launch per "
               "pattern; a step counts one of 20 strided slices of every pattern's root edges, so "
               "20 steps count every embedding once; patterns whose tuned full run is estimated "
               "above --max-pattern-s are reported with their estimate, not run", "sliced"),
    "list-rmat17": (1, ["5-clique"],
                    "R-MAT scale 17, edge factor 8, (0.57,0.19,0.19,0.05), seed 2; every 5-clique "
                    "listed (original vertex ids, one row per subgraph) into a buffer resident in HBM",
                    "list"),
    "iep-rmat17": (1, ["k4-path", "house"],
                   "R-MAT scale 17, edge factor 8, (0.57,0.19,0.19,0.05), seed 2; K4 plus a pendant "
                   "path and house counted with inclusion-exclusion over the last two levels, one "
                   "launch each, against plain counting", "iep"),
    "serve": (None, None,
              "serving: R-MAT-17, Chung-Lu 7000 and R-MAT-22 resident; Poisson stream of 2,000 "
              "queries at 50 QPS, seed 5, each a uniform draw from the 141 connected 3-6-vertex "
              "pattern classes on a uniform graph", "serve"),
}


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--slices", type=int, default=20,
                    help="sliced workloads: a step counts one of this many strided root slices")
    ap.add_argument("--traffic-slices", type=int, default=2,
                    help="sliced workloads: byte accounting of the batched launch on this many of "
                         "the timed slices")
    ap.add_argument("--patterns", default=None,
                    help="comma-separated subset of the workload's patterns (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-traffic", action="store_true",
                    help="skip the instrumented algorithmic-bytes run")
    ap.add_argument("--tune-seconds", type=float, default=8.0,
                    help="GPU-time budget per pattern for measured configuration selection")
    ap.add_argument("--plans-json", default=None,
                    help="reuse the configurations and launch shapes of a previous bench JSON "
                         "line instead of tuning (so profiled runs time the same kernels)")
    ap.add_argument("--traffic-json", default=None,
                    help="HBM bytes per launch from rocprofv3 counters (used only while the "
                         "kernel sources it was taken from are unchanged; default "
                         "profiles/traffic_<workload>.json)")
    ap.add_argument("--no-try-iep", action="store_true",
                    help="plain workloads: tune without inclusion-exclusion configurations")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the model's configurations and the default launch shape")
    ap.add_argument("--max-pattern-s", type=float, default=90.0,
                    help="batched workloads: patterns whose full run is estimated above this are "
                         "reported with their extrapolation instead of run")
    ap.add_argument("--batch-group", type=int, default=0,
                    help="lanes per group of the batched launch (0: measured by gp_batch_tune)")
    ap.add_argument("--batch-leaf", type=int, default=3)
    ap.add_argument("--queries", type=int, default=2000, help="serve: stream length")
    ap.add_argument("--qps", type=float, default=50.0, help="serve: mean arrival rate")
    ap.add_argument("--serve-leaf", type=int, default=1, help="serve: leaf mode of the batched launches")
    ap.add_argument("--max-query-ms", type=float, default=20.0,
                    help="serve: reject queries whose measured estimate exceeds this")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    return ap.parse_args()


_T0 = time.perf_counter()


def note(msg: str) -> None:
    print(f"[bench +{time.perf_counter() - _T0:.0f}s] {msg}", file=sys.stderr, flush=True)


def host_info() -> dict:
    """CPU model and counts of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


def oracle_threads() -> int:
    """Threads for the oracle: every CPU this process may use, within the
    16-CPU share a one-GPU machine allots to its GPU."""
    return max(1, min(16, host_info()["cpus_allowed"]))


def oracle_worker(folder: str) -> None:
    """Child process of cpu_baseline: counts the jobs read from stdin (one JSON
    list per line) with the oracle on one thread, one line out per job."""
    import numpy as np
    import oracle as O

    lay = O._CSRView(np.load(os.path.join(folder, "row_ptr.npy"), mmap_mode="r"),
                     np.load(os.path.join(folder, "col.npy"), mmap_mode="r"))
    print("ready", flush=True)
    for line in sys.stdin:
        k, e, restr, pins = json.loads(line)
        t = time.perf_counter()
        c = O.count_maps(lay, k, [tuple(x) for x in e], restr=[tuple(x) for x in restr],
                         pins=[tuple(x) for x in pins], threads=1)
        print(f"{c} {time.perf_counter() - t:.6f}", flush=True)


def cpu_baseline(g, plans, names, budget_s: float, threads: int | None = None,
                 job_limit_s: float | None = None) -> dict:
    """The oracle, untuned, on a bounded sample of the same workload: random
    root edges of each plan (in the oracle's own degree-sorted relabelling),
    each counted by the oracle with the first two schedule vertices pinned, in
    `threads` worker processes. New jobs start until the budget is spent; a job
    still running after job_limit_s is abandoned (its process killed), since
    one hub root can hold more work than the whole budget. The rate is the
    embeddings of the finished jobs over their summed one-thread time, times
    the threads."""
    import selectors
    import subprocess
    import tempfile
    import numpy as np
    import oracle as O

    rp, col, _ = O.relabel_by_degree(g)
    src = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    threads = threads or oracle_threads()
    job_limit_s = job_limit_s or max(1.0, budget_s / 2)
    rng = np.random.default_rng(12345)
    jobs = []
    for name, plan in zip(names, plans):
        order = plan.order
        restr = [list(x) for x in plan.restrictions]
        k, e = plan.k, [list(x) for x in plan.edges]
        cut = 1 if (order[0], order[1]) in plan.restrictions else (2 if (order[1], order[0]) in plan.restrictions else 0)
        ok = np.ones(len(col), bool) if cut == 0 else ((col < src) if cut == 1 else (col > src))
        cand = np.nonzero(ok)[0]
        for idx in rng.choice(cand, size=min(4000, cand.size), replace=False):
            jobs.append([k, e, restr, [[order[0], int(src[idx])], [order[1], int(col[idx])]]])
    rng.shuffle(jobs)

    folder = tempfile.mkdtemp(prefix="gp_oracle_")
    np.save(os.path.join(folder, "row_ptr.npy"), np.asarray(rp, dtype=np.int64))
    np.save(os.path.join(folder, "col.npy"), np.asarray(col, dtype=np.int32))
    del src
    sel = selectors.DefaultSelector()
    workers = {}  # pid -> [proc, job start time or None]

    def spawn():
        p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", folder],
                             stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, bufsize=1,
                             env=dict(os.environ, OMP_NUM_THREADS="1"))
        if p.stdout.readline().strip() != "ready":
            p.kill()
            p.wait()
            raise RuntimeError("oracle worker failed to start")
        workers[p.pid] = [p, None]
        sel.register(p.stdout, selectors.EVENT_READ, p.pid)
        return p

    def stop(pid, kill):
        p = workers.pop(pid)[0]
        sel.unregister(p.stdout)
        if kill:
            p.kill()
        else:
            p.stdin.close()
        p.wait()

    found = done = abandoned = 0
    busy = 0.0
    it = iter(jobs)
    try:
        for _ in range(threads):
            spawn()
        t0 = time.perf_counter()
        deadline = t0 + budget_s

        def feed(pid):
            j = next(it, None) if time.perf_counter() < deadline else None
            if j is None:
                stop(pid, kill=False)
                return
            workers[pid][0].stdin.write(json.dumps(j) + "\n")
            workers[pid][0].stdin.flush()
            workers[pid][1] = time.perf_counter()

        for pid in list(workers):
            feed(pid)
        while workers:
            for key, _ in sel.select(timeout=0.2):
                pid = key.data
                line = workers[pid][0].stdout.readline().split()
                if len(line) != 2:
                    raise RuntimeError("oracle worker ended early")
                found += int(line[0])
                busy += float(line[1])
                done += 1
                feed(pid)
            now = time.perf_counter()
            for pid in [q for q, (_, ts) in workers.items() if ts is not None and now - ts > job_limit_s]:
                stop(pid, kill=True)
                abandoned += 1
                if now < deadline:
                    feed(spawn().pid)
        wall = time.perf_counter() - t0
    finally:
        for pid in list(workers):
            stop(pid, kill=True)
        for f in ("row_ptr.npy", "col.npy"):
            os.remove(os.path.join(folder, f))
        os.rmdir(folder)
    value = found / busy * threads if busy > 0 else 0.0
    out = {"value": value, "unit": "embeddings/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} root edges drawn uniformly from the {len(plans)} plans' root tasks, each "
                     f"counted by the CPU oracle (one thread per job) with the first two schedule "
                     f"vertices pinned; {found} embeddings in {busy:.1f} s of summed job time, "
                     f"rate x {threads} worker processes ({wall:.1f} s wall); {abandoned} jobs "
                     f"abandoned after {job_limit_s:g} s each and left out of both sums",
           "jobs_done": done, "jobs_abandoned": abandoned, "wall_s": wall}
    out.update(host_info())
    return out


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the multi-GPU "
              "design replicates the graph and shards root edges, but this build runs on one GPU)",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import torch
    from paper_2009_10955_amd import gp
    from paper_2009_10955_amd import inputs as I

    torch.cuda.set_device(0)
    cfg_idx, names, desc, mode = WORKLOADS[args.workload]
    if args.traffic_json is None:
        args.traffic_json = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
    if mode == "serve":
        return serve_main(args, desc)
    if args.patterns:
        names = [n for n in names if n in args.patterns.split(",")]
    if mode == "sliced":
        return sliced_main(args, cfg_idx, names, desc)
    g = I.config_graph(cfg_idx)
    graph = gp.Graph.from_csr(g, device=True)
    st = graph.stats()
    t_plan = time.perf_counter()
    base_plans = [gp.Plan(*I.PATTERNS[n], stats=st, iep=(mode == "iep")) for n in names]
    plan_s = time.perf_counter() - t_plan
    t_tune = time.perf_counter()
    if args.plans_json:
        prev = json.loads(open(args.plans_json).read().strip().splitlines()[-1])["plans"]
        launches = [dict(prev[n]["launch"]) for n in names]
        # each plan carries its recorded launch shape (the one a batch runs it at)
        plans = [gp.Plan(*I.PATTERNS[n], stats=st, force_order=prev[n]["order"],
                         force_restr=[tuple(x) for x in prev[n]["restrictions"]],
                         iep=int(prev[n].get("iep", mode == "iep"))).with_launch(**l)
                 for n, l in zip(names, launches)]
    elif args.no_tune:
        plans = base_plans
        launches = [p.launch() for p in plans]
    else:
        plans = []
        for n, p in zip(names, base_plans):
            plans.append(p.tuned(graph, budget_seconds=args.tune_seconds,
                                 try_iep=(mode == "plain" and not args.no_try_iep)))
            note(f"tuned {n}")
        launches = [p.launch() for p in plans]
    tune_s = time.perf_counter() - t_tune
    if mode == "batched":
        return batched_main(args, desc, g, graph, st, names, plans, launches, base_plans, plan_s, tune_s)
    if mode == "list":
        return list_main(args, desc, g, graph, st, names, plans, launches, base_plans, plan_s, tune_s)
    stream = torch.cuda.current_stream()
    dev_out = torch.zeros(2 * len(plans), dtype=torch.int64, device="cuda")

    note(f"graph loaded: n={st.n} m={st.m} max_degree={st.max_degree} hubs={st.hub_vertices} "
         f"load={st.load_seconds:.3f}s plan={plan_s:.2f}s tune={tune_s:.1f}s; plans: " +
         ", ".join(f"{n} {p.order} {p.restrictions} {l}" for n, p, l in zip(names, plans, launches)))

    def step(events=None):
        for i, (p, l) in enumerate(zip(plans, launches)):
            if events is not None:
                events[i][0].record(stream)
            gp.count_async(graph, p, dev_out[2 * i:2 * i + 2], stream, **l)
            if events is not None:
                events[i][1].record(stream)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        note(f"warmup step {w + 1}/{args.warmup} done")

    per_kernel = [[] for _ in plans]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in plans] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(args.steps):
        step(evs[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    note(f"{args.steps} timed steps done: {ms_total / args.steps:.1f} ms/step")
    for s in range(args.steps):
        for i in range(len(plans)):
            per_kernel[i].append(evs[s][i][0].elapsed_time(evs[s][i][1]))
    res = dev_out.cpu().tolist()
    counts = [res[2 * i] & (2 ** 64 - 1) for i in range(len(plans))]
    flags = [res[2 * i + 1] for i in range(len(plans))]
    if any(flags):
        raise RuntimeError(f"count flags (1: overflow, 2: internal): {dict(zip(names, flags))}")
    ms_per_step = ms_total / args.steps
    embeddings_per_step = sum(counts)
    value = embeddings_per_step / (ms_per_step / 1e3)

    avg_ms = [sum(x) / len(x) for x in per_kernel]
    dom = max(range(len(plans)), key=lambda i: avg_ms[i])
    roofline = None
    alg = {}
    if not args.no_traffic:
        for i, (n, p, l) in enumerate(zip(names, plans, launches)):
            c, b = gp.count_traffic(graph, p, **l)
            assert c == counts[i]
            alg[n] = b
            note(f"algorithmic bytes {n}: {b:.4e}")
        achieved = alg[names[dom]] / (avg_ms[dom] / 1e3) / 1e9
        traffic = None
        from paper_2009_10955_amd import profiling
        tr = profiling.load_traffic(args.traffic_json)
        dom_plan = {"order": list(plans[dom].order),
                    "restrictions": [list(x) for x in plans[dom].restrictions],
                    "launch": launches[dom], "iep": bool(plans[dom].info().iep)}
        l2 = None
        src = None
        if (tr is not None and tr["pattern"] == names[dom] and tr["workload"] == args.workload
                and profiling.same_plan(tr.get("plan"), dom_plan)):
            traffic = tr["hbm_bytes_per_launch"]
            l2 = tr.get("l2")
            src = os.path.relpath(args.traffic_json, ROOT)
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                    "traffic_source": src,
                    "kernel": f"count_kernel ({names[dom]})",
                    "alg_bytes_per_launch": alg[names[dom]],
                    "avg_launch_ms": round(avg_ms[dom], 3),
                    "dram_GBps": round(traffic / (avg_ms[dom] / 1e3) / 1e9, 2) if traffic else None,
                    "l2_hit_rate": round(l2["hit_rate"], 5) if l2 else None}

    if args.copy_mib > 0:
        x = torch.empty(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    plain = None
    if mode == "iep":
        # the same patterns counted without inclusion-exclusion, each tuned
        plain = {}
        for i, (n, b) in enumerate(zip(names, base_plans)):
            pp = gp.Plan(*I.PATTERNS[n], stats=st)
            if not args.no_tune and not args.plans_json:
                pp = pp.tuned(graph, budget_seconds=args.tune_seconds)
            pl = pp.launch()
            ts = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                gp.count_async(graph, pp, dev_out[2 * i:2 * i + 2], stream, **pl)
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            c = int(dev_out[2 * i].item())
            if c != counts[i]:
                raise RuntimeError(f"{n}: plain count {c} != IEP count {counts[i]}")
            plain[n] = {"kernel_ms": round(min(ts), 3), "iep_speedup": round(min(ts) / avg_ms[i], 3),
                        "iep": bool(plans[i].info().iep), "launch": pl}
            note(f"plain {n}: {min(ts):.2f} ms (IEP {avg_ms[i]:.2f} ms)")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, plans, names, args.cpu_seconds)
        note(f"cpu baseline: {cpu['value']:.4e} embeddings/s on {cpu['cores']} threads")
        one = cpu_baseline(g, plans, names, args.cpu_seconds / 2, threads=1)
        cpu["value_1_thread"] = one["value"]
        cpu["sample_1_thread"] = one["sample"]
        note(f"cpu baseline, 1 thread: {one['value']:.4e} embeddings/s")

    out = {
        "metric": METRIC if mode != "iep" else "embeddings/s counted with inclusion-exclusion",
        "value": value,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "graph": {"n": st.n, "m": st.m, "max_degree": st.max_degree,
                                               "sha256": g.sha256()},
                   "patterns": names, "parallelism": "single GPU"},
        "counts": dict(zip(names, counts)),
        "kernel_ms": {n: round(a, 3) for n, a in zip(names, avg_ms)},
        "intersection_GBps": {n: round(alg[n] / (a / 1e3) / 1e9, 2) for n, a in zip(names, avg_ms)}
        if alg else None,
        "plans": {n: {"order": list(p.order), "restrictions": [list(x) for x in p.restrictions],
                      "launch": l, "iep": bool(p.info().iep), "model_order": list(b.order),
                      "model_restrictions": [list(x) for x in b.restrictions]}
                  for n, p, b, l in zip(names, plans, base_plans, launches)},
        "preprocessing_s": {"load": st.load_seconds, "plan": plan_s, "tune": tune_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if plain is not None:
        out["plain"] = plain
    print(json.dumps(out), flush=True)


def list_main(args, desc, g, graph, st, names, plans, launches, base_plans, plan_s, tune_s):
    """Listing: every embedding written as a row of k original vertex ids into
    one preallocated device buffer; a step is one gp_list call per pattern."""
    import numpy as np
    import torch
    from paper_2009_10955_amd import gp
    stream = torch.cuda.current_stream()
    counts = [gp.count(graph, p, **l) for p, l in zip(plans, launches)]
    bufs = [torch.empty((max(1, c), p.k), dtype=torch.int32, device="cuda") for p, c in zip(plans, counts)]
    note("listing " + ", ".join(f"{n}: {c} rows ({c * p.k * 4 / 1e9:.2f} GB)"
                                for n, p, c in zip(names, plans, counts)))
    lists = [dict(l, group=0, leaf_mode=0) for l in launches]

    def step(events=None):
        for i, (p, l) in enumerate(zip(plans, lists)):
            if events is not None:
                events[i][0].record(stream)
            _, total = gp.list_embeddings(graph, p, capacity=counts[i], out=bufs[i], stream=stream, **l)
            if total != counts[i]:
                raise RuntimeError(f"{names[i]}: listed {total}, counted {counts[i]}")
            if events is not None:
                events[i][1].record(stream)

    for w in range(args.warmup):
        step()
        note(f"warmup step {w + 1}/{args.warmup} done")
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in plans] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    per = [[evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(args.steps)] for i in range(len(plans))]
    avg_ms = [sum(x) / len(x) for x in per]
    note(f"{args.steps} timed steps done: {ms_per_step:.1f} ms/step")

    # sampled validity of the rows of the last step: injective, every pattern
    # edge on a data edge (original ids)
    rng = np.random.default_rng(0)
    n = g.row_ptr.shape[0] - 1
    adj = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr)) * n + np.asarray(g.col, np.int64)
    for i, (name, p) in enumerate(zip(names, plans)):
        if counts[i] == 0:
            continue
        idx = torch.from_numpy(rng.integers(0, counts[i], 100_000)).cuda()
        rows = bufs[i][idx].cpu().numpy().astype(np.int64)
        assert (np.diff(np.sort(rows, axis=1), axis=1) > 0).all(), name
        for a, b in p.edges:
            assert np.isin(rows[:, a] * n + rows[:, b], adj).all(), name

    dom = max(range(len(plans)), key=lambda i: avg_ms[i])
    roofline = None
    alg = {}
    if not args.no_traffic:
        for i, (name, p, l) in enumerate(zip(names, plans, launches)):
            c, b = gp.count_traffic(graph, p, **l)
            assert c == counts[i]
            alg[name] = b + 4 * p.k * counts[i]
            note(f"algorithmic bytes {name}: search {b:.4e} + rows {4 * p.k * counts[i]:.4e}")
        achieved = alg[names[dom]] / (avg_ms[dom] / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                    "kernel": f"list_kernel ({names[dom]})", "alg_bytes_per_launch": alg[names[dom]],
                    "avg_launch_ms": round(avg_ms[dom], 3),
                    "rows_GBps": round(4 * plans[dom].k * counts[dom] / (avg_ms[dom] / 1e3) / 1e9, 2)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, plans, names, args.cpu_seconds)
        cpu["sample"] += " (counted, not listed)"
        note(f"cpu baseline: {cpu['value']:.4e} embeddings/s on {cpu['cores']} threads")
    out = {
        "metric": "embeddings listed/s",
        "value": sum(counts) / (ms_per_step / 1e3),
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "graph": {"n": st.n, "m": st.m, "max_degree": st.max_degree,
                                               "sha256": g.sha256()},
                   "patterns": names, "parallelism": "single GPU"},
        "counts": dict(zip(names, counts)),
        "kernel_ms": {name: round(a, 3) for name, a in zip(names, avg_ms)},
        "plans": {name: {"order": list(p.order), "restrictions": [list(x) for x in p.restrictions],
                         "launch": l} for name, p, l in zip(names, plans, lists)},
        "preprocessing_s": {"load": st.load_seconds, "plan": plan_s, "tune": tune_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def batched_main(args, desc, g, graph, st, names, plans, launches, base_plans, plan_s, tune_s):
    """Batched workloads: the feasible patterns counted by one batch
    (replayed from a hipGraph), against one launch per pattern (each its own
    launch and synchronisation), at identical counts."""
    import torch
    from paper_2009_10955_amd import gp

    stream = torch.cuda.current_stream()
    infeasible = {}
    keep = []
    for i, (n, p, l) in enumerate(zip(names, plans, launches)):
        if p.info().iep:
            keep.append(i)
            continue
        e = gp.estimate(graph, p, budget_ms=args.max_pattern_s * 1e3, stream=stream, **l)
        note(f"estimate {n}: {e['ms'] / 1e3:.2f} s (sample 1/{e['sample_stride']}: "
             f"{e['sample_count']} embeddings)")
        if e["ms"] > args.max_pattern_s * 1e3:
            infeasible[n] = {"estimated_s": None if e["ms"] == float("inf") else e["ms"] / 1e3,
                             "estimate_note": "a wavefront of the root sample alone ran past the "
                                              "limit" if e["ms"] == float("inf") else
                                              "wavefront busy time of the root sample, scaled",
                             "sample_stride": e["sample_stride"],
                             "sample_count": e["sample_count"],
                             "count_extrapolated": e["sample_count"] * e["sample_stride"]}
        else:
            keep.append(i)
    names = [names[i] for i in keep]
    plans = [plans[i] for i in keep]
    launches = [launches[i] for i in keep]
    base_plans = [base_plans[i] for i in keep]
    if not plans:
        raise SystemExit("no pattern of the workload is feasible within --max-pattern-s")
    if args.batch_group > 0:
        blaunch = dict(group=args.batch_group, leaf_mode=args.batch_leaf)
    else:
        blaunch, bms = gp.batch_tune(graph, plans, stream)
        note(f"batch shape {blaunch}: {bms:.1f} ms")
    batch = gp.Batch(graph, plans, stream, **blaunch)

    plain_each = [[] for _ in plans]

    def plain_step():
        out = []
        for i, (p, l) in enumerate(zip(plans, launches)):
            t = time.perf_counter()
            out.append(gp.count(graph, p, stream, **l))
            plain_each[i].append((time.perf_counter() - t) * 1e3)
        return out

    for w in range(args.warmup):
        batch.run(stream)
        plain_step()
        note(f"warmup {w + 1}/{args.warmup} done")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    b_ms, p_ms = [], []
    counts_b = counts_p = None
    for s in range(args.steps):
        a, b = ev(), ev()
        torch.cuda.synchronize()
        a.record(stream)
        counts_b = batch.run(stream)
        b.record(stream)
        torch.cuda.synchronize()
        b_ms.append(a.elapsed_time(b))
        a, b = ev(), ev()
        a.record(stream)
        counts_p = plain_step()
        b.record(stream)
        torch.cuda.synchronize()
        p_ms.append(a.elapsed_time(b))
        note(f"step {s + 1}/{args.steps}: batched {b_ms[-1]:.1f} ms, plain {p_ms[-1]:.1f} ms")
    if counts_b != counts_p:
        raise RuntimeError(f"batched counts {counts_b} differ from plain counts {counts_p}")
    # like for like: one launch per pattern at the batch's own launch shape
    same_ms = []
    for s in range(args.steps):
        a, b = ev(), ev()
        torch.cuda.synchronize()
        a.record(stream)
        counts_s = [gp.count(graph, p, stream, **dict(l, **blaunch)) for p, l in zip(plans, launches)]
        b.record(stream)
        torch.cuda.synchronize()
        same_ms.append(a.elapsed_time(b))
    if counts_s != counts_b:
        raise RuntimeError("plain counts at the batch's shape differ")
    note(f"plain at the batch's shape: {sum(same_ms) / len(same_ms):.1f} ms per step")
    ms_b = sum(b_ms) / len(b_ms)
    ms_p = sum(p_ms) / len(p_ms)
    value = sum(counts_b) / (ms_b / 1e3)
    roofline = None
    if not args.no_traffic:
        alg = 0
        for n, p, l, c in zip(names, plans, launches, counts_b):
            cc, bb = gp.count_traffic(graph, p, **l)
            assert cc == c
            alg += bb
        achieved = alg / (ms_b / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                    "kernel": "the batch's launches (all feasible patterns, one hipGraph replay)",
                    "alg_bytes_per_launch": alg, "avg_launch_ms": round(ms_b, 3)}
    cpu = None
    if not args.no_cpu_baseline and args.workload != "rmat22":
        cpu = cpu_baseline(g, plans, names, args.cpu_seconds)
    out = {
        "metric": METRIC, "value": value, "unit": "embeddings/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": desc, "graph": {"n": st.n, "m": st.m, "max_degree": st.max_degree,
                                               "sha256": g.sha256()},
                   "patterns": names, "parallelism": "single GPU",
                   "batch_launch": blaunch},
        "counts": dict(zip(names, counts_b)),
        "plain_ms_per_step": ms_p,
        "plain_same_shape_ms_per_step": sum(same_ms) / len(same_ms),
        "batched_speedup_same_shape": (sum(same_ms) / len(same_ms)) / ms_b,
        "plain_ms_per_pattern": {n: round(sum(x[-args.steps:]) / len(x[-args.steps:]), 3)
                                 for n, x in zip(names, plain_each)},
        "batched_speedup": ms_p / ms_b,
        "batched_ms": b_ms, "plain_ms": p_ms,
        "infeasible": infeasible,
        "plans": {n: {"order": list(p.order), "restrictions": [list(x) for x in p.restrictions],
                      "launch": l, "model_order": list(b.order),
                      "model_restrictions": [list(x) for x in b.restrictions]}
                  for n, p, b, l in zip(names, plans, base_plans, launches)},
        "preprocessing_s": {"load": st.load_seconds, "plan": plan_s, "tune": tune_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def sliced_main(args, cfg_idx, names, desc):
    """The batched configuration at scale. Every pattern is planned, its full
    run estimated, tuned (IEP configurations competing) and estimated again;
    those above --max-pattern-s are reported with their estimate. A step
    counts slice s (root edges s, s + S, s + 2S, ... of every feasible
    pattern, heavy roots split as tuned) with the batched launches replayed
    from a hipGraph; the same slices are then counted with one launch per
    pattern. S steps count every embedding once."""
    import torch
    from paper_2009_10955_amd import gp
    from paper_2009_10955_amd import inputs as I

    S = max(1, args.slices)
    t0 = time.perf_counter()
    g = I.config_graph(cfg_idx)
    note(f"graph generated in {time.perf_counter() - t0:.1f} s: n={g.n} m={g.m}")
    graph = gp.Graph.from_csr(g, device=True)
    st = graph.stats()
    stream = torch.cuda.current_stream()
    t_plan = time.perf_counter()
    base_plans = [gp.Plan(*I.PATTERNS[n], stats=st) for n in names]
    plan_s = time.perf_counter() - t_plan
    plans, launches, keep, infeasible = [], [], [], {}
    t_tune = time.perf_counter()
    for n, bp in zip(names, base_plans):
        e0 = gp.estimate(graph, bp, budget_ms=min(30.0, args.max_pattern_s) * 1e3, stream=stream)
        note(f"{n}: model plan estimated at {e0['ms'] / 1e3:.1f} s")
        if e0["ms"] > 10 * args.max_pattern_s * 1e3:
            infeasible[n] = {"estimated_s": None if e0["ms"] == float("inf") else e0["ms"] / 1e3,
                             "of": "the model's configuration, default launch",
                             "count_extrapolated": e0["sample_count"] * e0["sample_stride"]}
            continue
        if args.plans_json:
            prev = json.loads(open(args.plans_json).read().strip().splitlines()[-1])["plans"][n]
            lt = dict(prev["launch"])
            tp = gp.Plan(*I.PATTERNS[n], stats=st, force_order=prev["order"],
                         force_restr=[tuple(x) for x in prev["restrictions"]],
                         iep=int(prev.get("iep", 0))).with_launch(**lt)
        else:
            tp = bp.tuned(graph, budget_seconds=args.tune_seconds, try_iep=not args.no_try_iep)
            lt = tp.launch()
        e1 = gp.estimate(graph, tp, budget_ms=args.max_pattern_s * 1e3, stream=stream, **lt)
        note(f"{n}: tuned {tp.order} {tp.restrictions} iep={tp.info().iep} {lt}: "
             f"estimated at {e1['ms'] / 1e3:.1f} s")
        if e1["ms"] > args.max_pattern_s * 1e3:
            infeasible[n] = {"estimated_s": None if e1["ms"] == float("inf") else e1["ms"] / 1e3,
                             "of": "the tuned configuration and launch",
                             "count_extrapolated": e1["sample_count"] * e1["sample_stride"]}
            continue
        keep.append(n)
        plans.append(tp)
        launches.append(lt)
    tune_s = time.perf_counter() - t_tune
    if not plans:
        raise SystemExit("no pattern of the workload is feasible within --max-pattern-s")
    names_all, names = names, keep
    batch = gp.Batch(graph, plans, stream)
    dev_out = torch.zeros(2 * len(plans), dtype=torch.int64, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def batched_step(s, events=None):
        batch.set_sample(S, s % S, stream)
        if events is not None:
            events[0].record(stream)
        c = batch.run(stream)
        if events is not None:
            events[1].record(stream)
        return c

    def plain_step(s, events=None):
        for i, (p, l) in enumerate(zip(plans, launches)):
            if events is not None:
                events[i][0].record(stream)
            gp.count_async(graph, p, dev_out[2 * i:2 * i + 2], stream, root_stride=S, root_offset=s % S, **l)
            if events is not None:
                events[i][1].record(stream)
        torch.cuda.synchronize()
        r = dev_out.cpu().tolist()
        return [r[2 * i] & (2 ** 64 - 1) for i in range(len(plans))]

    for w in range(args.warmup):
        batched_step(w)
        plain_step(w)
        note(f"warmup step {w + 1}/{args.warmup} done")
    if args.copy_mib > 0:
        # a plain device copy of known size: calibrates the traffic counters
        x = torch.empty(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    # batched: K steps
    b_ev = [(ev(), ev()) for _ in range(args.steps)]
    counts_b = []
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    for s in range(args.steps):
        counts_b.append(batched_step(s, b_ev[s]))
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - tb0) * 1e3
    note(f"{args.steps} batched steps: {ms_b / args.steps:.1f} ms/step")
    # plain: the same K slices, one launch per pattern
    p_ev = [[(ev(), ev()) for _ in plans] for _ in range(args.steps)]
    counts_p = []
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for s in range(args.steps):
        counts_p.append(plain_step(s, p_ev[s]))
    torch.cuda.synchronize()
    ms_p = (time.perf_counter() - tp0) * 1e3
    note(f"{args.steps} plain steps: {ms_p / args.steps:.1f} ms/step")
    if counts_b != counts_p:
        raise RuntimeError(f"batched counts differ from plain counts: {counts_b} vs {counts_p}")
    launch_ms = [b_ev[s][0].elapsed_time(b_ev[s][1]) for s in range(args.steps)]
    kernel_ms = {n: round(sum(p_ev[s][i][0].elapsed_time(p_ev[s][i][1]) for s in range(args.steps)) /
                          args.steps, 3) for i, n in enumerate(names)}
    emb = sum(sum(c) for c in counts_b)
    value = emb / (ms_b / 1e3)
    # totals: the timed slices cover every root once when K is a multiple of S
    whole = args.steps % S == 0
    totals = {n: sum(c[i] for c in counts_b[:S]) for i, n in enumerate(names)} if args.steps >= S else None

    roofline = None
    if not args.no_traffic:
        # bytes of the batched launch on the first timed slices: the same
        # slices, plans and launches through the instrumented kernel
        nt = max(1, min(args.traffic_slices, args.steps))
        alg = 0
        for s in range(nt):
            for i, (p, l) in enumerate(zip(plans, launches)):
                c, b = gp.count_traffic(graph, p, root_stride=S, root_offset=s % S, **l)
                if c != counts_b[s][i]:
                    raise RuntimeError(f"accounting count {c} != {counts_b[s][i]} ({names[i]}, slice {s})")
                alg += b
            note(f"byte accounting, slice {s}: {alg:.4e} B so far")
        t_acc = sum(launch_ms[:nt]) / 1e3
        achieved = alg / t_acc / 1e9
        from paper_2009_10955_amd import profiling
        tr = profiling.load_traffic(args.traffic_json) if args.traffic_json else None
        traffic = None
        src = None
        cur = {n: {"order": list(p.order), "restrictions": [list(x) for x in p.restrictions],
                   "launch": l, "iep": bool(p.info().iep)} for n, p, l in zip(names, plans, launches)}
        # the counters were taken on the longest launch of the step: they apply
        # while that pattern's plan and launch are the same
        dom = max(names, key=lambda n: kernel_ms[n])
        if (tr is not None and tr.get("workload") == args.workload
                and tr.get("kernel_match") in ("batch_kernel", "count_kernel")
                and isinstance(tr.get("plan"), dict) and dom in tr["plan"]
                and profiling.same_plan(tr["plan"][dom], cur[dom])):
            traffic = tr["hbm_bytes_per_launch"]
            src = os.path.relpath(args.traffic_json, ROOT)
        l2 = tr.get("l2") if traffic is not None else None
        avg_ms = sum(launch_ms[:nt]) / nt
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                    "traffic_source": src,
                    "dram_GBps": round(traffic / (avg_ms / 1e3) / 1e9, 2) if traffic else None,
                    "l2_hit_rate": round(l2["hit_rate"], 5) if l2 else None,
                    "kernel": "the batched step's launches (one per plan shape; a shape with one plan "
                              "runs count_kernel, several share batch_kernel)",
                    "alg_bytes_per_launch": alg / nt, "alg_bytes_slices": nt,
                    "avg_launch_ms": round(sum(launch_ms[:nt]) / nt, 3),
                    "avg_launch_ms_all_steps": round(sum(launch_ms) / len(launch_ms), 3)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, plans, names, args.cpu_seconds)
        note(f"cpu baseline: {cpu['value']:.4e} embeddings/s on {cpu['cores']} threads")
    out = {
        "metric": METRIC, "value": value, "unit": "embeddings/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "graph": {"n": st.n, "m": st.m, "max_degree": st.max_degree,
                                               "sha256": g.sha256()},
                   "patterns": names, "patterns_reported_not_run": sorted(infeasible),
                   "slices": S, "parallelism": "single GPU"},
        "embeddings_per_step": emb / args.steps,
        "counts": totals, "counts_cover_every_root": bool(totals) and whole,
        # an IEP plan's slice counts are its slice totals divided by the
        # over-count, rounded down: their sum may fall short by under one per slice
        "counts_rounded_per_slice": [n for n, p in zip(names, plans) if p.info().iep_div > 1],
        "plain_ms_per_step": ms_p / args.steps,
        "batched_speedup": ms_p / ms_b,
        "batched_launch_ms": [round(x, 3) for x in launch_ms],
        "plain_kernel_ms_per_step": kernel_ms,
        "infeasible": infeasible,
        "plans": {n: {"order": list(p.order), "restrictions": [list(x) for x in p.restrictions],
                      "launch": l, "iep": int(p.info().iep), "iep_div": int(p.info().iep_div),
                      "tuned_ms": p.info().tuned_ms}
                  for n, p, l in zip(names, plans, launches)},
        "preprocessing_s": {"load": st.load_seconds, "plan": plan_s, "tune_and_estimates": tune_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    batch.close()
    print(json.dumps(out), flush=True)


def serve_main(args, desc):
    """Serving: replay a Poisson stream of queries against resident graphs
    through the continuous-batching server; every completed count is checked
    against a solo count of the same query."""
    from paper_2009_10955_amd import gp
    from paper_2009_10955_amd import inputs as I
    from paper_2009_10955_amd import serve as SV

    graphs, meta = [], []
    for ci in (1, 2, 3):
        g = I.config_graph(ci)
        G = gp.Graph.from_csr(g, device=True)
        s = G.stats()
        graphs.append(G)
        meta.append({"config": ci, "n": s.n, "m": s.m, "max_degree": s.max_degree,
                     "sha256": g.sha256()})
        note(f"graph {ci} resident: n={s.n} m={s.m}")
        del g
    classes = I.connected_patterns(3, 6)
    stream = I.poisson_stream(args.queries, args.qps, len(graphs), len(classes), seed=5)
    server = gp.Server(graphs, max_query_ms=args.max_query_ms, leaf_mode=args.serve_leaf)
    res = SV.run_stream(server, stream, classes, note=note)
    stats = server.stats()
    server.close()
    summ = SV.summarise(res)
    note(f"stream done: {summ}")
    # every completed query again, alone: one launch and synchronisation
    # each, in arrival order; its count must equal the served one
    import torch
    solo = {}
    plans_solo = {}
    bad = 0
    solo_s = 0.0
    t_last = time.perf_counter()
    for r in res:
        if time.perf_counter() - t_last > 10.0:
            t_last = time.perf_counter()
            note(f"solo runs: {len(solo)} distinct queries counted")
        if r["status"] != 0:
            continue
        key = (r["graph"], r["pattern"])
        G = graphs[r["graph"]]
        if key not in plans_solo:
            k, e = classes[r["pattern"]]
            plans_solo[key] = gp.Plan(k, e, stats=G.stats())
        torch.cuda.synchronize()
        t = time.perf_counter()
        c = gp.count(G, plans_solo[key])
        solo_s += time.perf_counter() - t
        solo[key] = c
        bad += c != r["count"]
    note(f"checked {sum(r['status'] == 0 for r in res)} completed counts against "
         f"{len(solo)} solo counts: {bad} mismatches")
    if bad:
        raise RuntimeError(f"{bad} served counts differ from their solo counts")
    out = {
        "metric": METRIC, "value": summ["completed"] / summ["wall_s"], "unit": "queries/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": summ["wall_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "graphs": meta, "queries": args.queries, "qps": args.qps,
                   "max_query_ms": args.max_query_ms, "leaf_mode": args.serve_leaf,
                   "parallelism": "single GPU"},
        "latency": summ,
        "server": stats,
        "solo_checked": len(solo), "mismatches": bad,
        "solo_total_s": solo_s,
        "served_gpu_s": stats["busy_seconds"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--oracle-worker":
        oracle_worker(sys.argv[2])
    else:
        main()
