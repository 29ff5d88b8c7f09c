"""Build libgp.so (the C-ABI library) in-tree with hipcc for gfx950."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgp.so")

# (source, extra defines, object name): the counting kernel is instantiated
# once per pattern size k, the batched kernel once per largest pattern size,
# each in its own unit so the variants build in parallel
SOURCES = [("api.cpp", [], "api.o"), ("planner.cpp", [], "planner.o"), ("tune.cpp", [], "tune.o"), ("server.cpp", [], "server.o"),
           ("graph.hip", [], "graph.o"), ("count.hip", [], "count.o"), ("list.hip", [], "list.o")] + [
    ("count_inst.hip", [f"-DGP_INST_K={k}"], f"count_k{k}.o") for k in range(2, 9)] + [
    ("count_batch.hip", [f"-DGP_BATCH_KMIN={a}", f"-DGP_BATCH_KMAX={b}"], f"count_batch_k{a}_{b}.o")
    for a, b in ((2, 2), (3, 3), (4, 4), (5, 5), (6, 6), (7, 8))]
ARCH = os.environ.get("GP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-ffp-contract=off",
        # no packed-FP32 instructions anywhere in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{INCLUDE}", f"-I{CSRC}",
        "-Wall", "-Wno-unused-result",
    ]


def _compile(item, verbose: bool) -> str:
    src, defines, oname = item
    obj = os.path.join(BUILD, oname)
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc()] + lang + ["-c", os.path.join(CSRC, src), "-o", obj] + defines + flags()
    if verbose:
        print(" ".join(cmd), flush=True)
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    if verbose:
        print(f"  {oname}: {time.time() - t:.1f}s", flush=True)
    return obj


def _stale(item) -> bool:
    """Whether an object is older than its source or any header."""
    src, _, oname = item
    obj = os.path.join(BUILD, oname)
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src), os.path.join(INCLUDE, "gp.h")] + [
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, jobs: int | None = None, changed_only: bool = False) -> str:
    """Compile every unit (changed_only: only those older than their sources)
    and link libgp.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 2)))
    todo = [s for s in SOURCES if _stale(s)] if changed_only else SOURCES
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [os.path.join(BUILD, o) for _, _, o in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, changed_only="--changed" in sys.argv))
