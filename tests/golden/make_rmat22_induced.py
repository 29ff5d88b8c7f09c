"""Write rmat22_induced.json: oracle counts on seeded induced subgraphs of the
R-MAT scale-22 graph (edge factor 8, a=0.57 b=0.19 c=0.19, seed 4), the
parity cases of that configuration that the CPU oracle finishes in seconds.

Each subgraph (inputs.core_subgraph) keeps the `hubs` highest-degree vertices
and `rest` seeded random others, induced on their union. Counts come from the
CPU oracle only.
Run from the repository root: python tests/golden/make_rmat22_induced.py
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2009_10955_amd import inputs as I  # noqa: E402

CASES = [
    # (name, hubs, rest, seed, patterns)
    ("core64", 64, 4000, 7, ["4-clique", "house", "5-cycle"]),
    ("core32", 32, 2000, 7, ["4-clique", "house", "5-cycle", "6-cycle-chord"]),
    ("core128", 128, 8000, 9, ["4-clique"]),
]


def main() -> None:
    g = I.config_graph(3)
    out = {"_about": "Oracle counts on induced subgraphs of the R-MAT scale-22 graph (configs[3] "
                     "parity); written by make_rmat22_induced.py, which calls only the CPU oracle.",
           "graph_sha256": g.sha256(), "cases": []}
    for name, hubs, rest, seed, pats in CASES:
        h = I.core_subgraph(g, hubs, rest, seed)
        case = {"name": name, "hubs": hubs, "rest": rest, "seed": seed, "n": h.n, "m": h.m,
                "sha256": h.sha256(), "counts": {}}
        for p in pats:
            t = time.time()
            case["counts"][p] = O.count(h, *I.PATTERNS[p], threads=8)
            print(f"{name} {p}: {case['counts'][p]} ({time.time() - t:.1f} s)", flush=True)
        out["cases"].append(case)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat22_induced.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
