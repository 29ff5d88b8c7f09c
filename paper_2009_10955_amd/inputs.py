"""Seeded synthetic inputs: data graphs as sorted int32 CSR, and query patterns.

This module is shared by the tests, the benchmark and the CPU oracle's callers.
It holds none of the counting method's arithmetic: it only draws graphs and
patterns from fixed seeds and puts edge lists into canonical CSR form
(symmetric, no self-loops, no duplicates, each neighbor list ascending).

The paper evaluates on public graphs (Wiki-Vote, MiCo, Patents, LiveJournal,
Orkut, Twitter; Section V, Table I). None of them is available here, so seeded
generators stand in with their shapes:

* ``er``       -- Erdos-Renyi G(n, p); the small exact-parity case.
* ``rmat``     -- R-MAT(a, b, c, d) power-law graphs (MiCo / LiveJournal sized).
* ``chung_lu`` -- Chung-Lu expected-degree graph with a power-law weight
  sequence (Wiki-Vote sized).

All generators use numpy's PCG64 ``default_rng(seed)`` with a fixed draw order,
so a (generator, parameters, seed) triple names one graph everywhere.
"""
from __future__ import annotations

import hashlib
import itertools
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class CSR:
    """Undirected simple graph as sorted CSR (both directions stored)."""

    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    """Canonical CSR of the undirected simple graph spanned by (src, dst).

    Symmetrises, drops self-loops and duplicate edges, sorts each list.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    key = np.unique(a * n + b)
    rows = key // n
    cols = (key % n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(row_ptr=row_ptr, col=cols)


def er(n: int = 1000, p: float = 0.01, seed: int = 1) -> CSR:
    """G(n, p): one Bernoulli(p) draw per pair i<j, in np.triu_indices order."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    return csr_from_edges(n, iu[keep], ju[keep])


def rmat(scale: int, edge_factor: int = 8, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 2, chunk: int = 1 << 22) -> CSR:
    """R-MAT graph on 2**scale vertices with edge_factor * 2**scale draws.

    Each draw picks one of four quadrants per level (probabilities a, b, c,
    d = 1-a-b-c), most significant bit first; no noise, no id permutation.
    The result is symmetrised with self-loops and duplicates removed.
    Draws are generated in fixed-size chunks, in order, so the graph does not
    depend on available memory.
    """
    n = 1 << scale
    total = edge_factor * n
    rng = np.random.default_rng(seed)
    cum = np.array([a, a + b, a + b + c], dtype=np.float64)
    keys = []
    done = 0
    while done < total:
        cnt = min(chunk, total - done)
        u = rng.random((cnt, scale))
        q = np.searchsorted(cum, u, side="right").astype(np.int64)  # 0..3
        weights = (1 << np.arange(scale - 1, -1, -1, dtype=np.int64))
        src = ((q >> 1) * weights).sum(axis=1)
        dst = ((q & 1) * weights).sum(axis=1)
        keep = src != dst
        src, dst = src[keep], dst[keep]
        lo = np.minimum(src, dst)
        hi = np.maximum(src, dst)
        keys.append(np.unique(lo * n + hi))
        done += cnt
    key = np.unique(np.concatenate(keys))
    return csr_from_edges(n, key // n, key % n)


def chung_lu(n: int = 7000, m_target: int = 100_000, gamma: float = 2.1,
             seed: int = 3, max_iter: int = 100) -> CSR:
    """Chung-Lu graph with power-law weights w_i ~ (i+1)^(-1/(gamma-1)).

    Weights are capped at sqrt(sum w) and rescaled until sum w = 2 m_target
    (without the cap, edge probabilities saturate at 1 and the graph falls
    well short of m_target). Edge (i, j), i<j, is kept with probability
    min(1, w_i w_j / sum w), drawn row by row.
    """
    rng = np.random.default_rng(seed)
    w = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
    target = 2.0 * m_target
    for _ in range(max_iter):
        w *= target / w.sum()
        cap = np.sqrt(target)
        if w.max() <= cap * (1 + 1e-12):
            break
        w = np.minimum(w, cap)
    total = w.sum()
    src_l, dst_l = [], []
    for i in range(n - 1):
        pr = np.minimum(1.0, w[i] * w[i + 1:] / total)
        hit = np.nonzero(rng.random(n - i - 1) < pr)[0]
        if hit.size:
            src_l.append(np.full(hit.size, i, dtype=np.int64))
            dst_l.append(hit.astype(np.int64) + i + 1)
    src = np.concatenate(src_l) if src_l else np.zeros(0, np.int64)
    dst = np.concatenate(dst_l) if dst_l else np.zeros(0, np.int64)
    return csr_from_edges(n, src, dst)


def gnm_small(n: int, p: float, seed: int) -> CSR:
    """Small G(n, p) for brute-force cross-checks (same draw order as ``er``)."""
    return er(n, p, seed)


def complete(n: int) -> CSR:
    i, j = np.triu_indices(n, 1)
    return csr_from_edges(n, i, j)


def complete_bipartite(a: int, b: int) -> CSR:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return csr_from_edges(a + b, i.ravel(), j.ravel())


def hypercube(d: int) -> CSR:
    n = 1 << d
    v = np.arange(n)
    src = np.concatenate([v for _ in range(d)])
    dst = np.concatenate([v ^ (1 << t) for t in range(d)])
    return csr_from_edges(n, src, dst)


def cycle_graph(n: int) -> CSR:
    v = np.arange(n)
    return csr_from_edges(n, v, (v + 1) % n)


def star(s: int) -> CSR:
    return csr_from_edges(s + 1, np.zeros(s, np.int64), np.arange(1, s + 1))


def disjoint_union(g: CSR, h: CSR) -> CSR:
    src_g = np.repeat(np.arange(g.n), g.degrees())
    src_h = np.repeat(np.arange(h.n), h.degrees()) + g.n
    src = np.concatenate([src_g, src_h])
    dst = np.concatenate([g.col.astype(np.int64), h.col.astype(np.int64) + g.n])
    return csr_from_edges(g.n + h.n, src, dst)


def permute(g: CSR, perm: np.ndarray) -> CSR:
    """Relabel vertex v as perm[v] (perm is a permutation of 0..n-1)."""
    src = np.repeat(np.arange(g.n), g.degrees())
    return csr_from_edges(g.n, perm[src], perm[g.col])


def induced_subgraph(g: CSR, keep: np.ndarray) -> CSR:
    """Subgraph induced on the sorted vertex set ``keep``, relabelled 0..|keep|-1."""
    keep = np.asarray(keep, dtype=np.int64)
    new_id = np.full(g.n, -1, dtype=np.int64)
    new_id[keep] = np.arange(keep.size)
    src = np.repeat(np.arange(g.n), g.degrees())
    dst = g.col.astype(np.int64)
    sel = (new_id[src] >= 0) & (new_id[dst] >= 0)
    return csr_from_edges(keep.size, new_id[src[sel]], new_id[dst[sel]])


def core_subgraph(g: CSR, hubs: int, rest: int, seed: int) -> CSR:
    """Seeded induced subgraph that keeps the `hubs` highest-degree vertices
    (ties: lower id first) and `rest` vertices drawn without replacement from
    the others (PCG64 default_rng(seed)), relabelled in ascending original id:
    a small piece of a power-law graph with its dense core."""
    order = np.argsort(-g.degrees(), kind="stable")
    rng = np.random.default_rng(seed)
    keep = np.sort(np.concatenate([order[:hubs], rng.choice(order[hubs:], rest, replace=False)]))
    return induced_subgraph(g, keep)


# ---------------------------------------------------------------- patterns
# Edge lists over vertices 0..k-1, as used by the evaluation configurations.

PATTERNS = {
    "triangle": (3, [(0, 1), (1, 2), (2, 0)]),
    "4-cycle": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "4-clique": (4, [(i, j) for i, j in itertools.combinations(range(4), 2)]),
    "house": (5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)]),
    "5-cycle": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]),
    "5-clique": (5, [(i, j) for i, j in itertools.combinations(range(5), 2)]),
    "6-cycle": (6, [(i, (i + 1) % 6) for i in range(6)]),
    "6-cycle-chord": (6, [(i, (i + 1) % 6) for i in range(6)] + [(0, 3)]),
    "prism": (6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3), (0, 3), (1, 4), (2, 5)]),
    "k4-path": (6, [(i, j) for i, j in itertools.combinations(range(4), 2)] + [(3, 4), (4, 5)]),
    "5-wheel": (6, [(i, (i + 1) % 5) for i in range(5)] + [(i, 5) for i in range(5)]),
    "6-clique": (6, [(i, j) for i, j in itertools.combinations(range(6), 2)]),
    "4-path": (4, [(0, 1), (1, 2), (2, 3)]),
    "3-star": (4, [(0, 1), (0, 2), (0, 3)]),
    "tailed-triangle": (4, [(0, 1), (1, 2), (2, 0), (2, 3)]),
    "diamond": (4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]),
    "edge": (2, [(0, 1)]),
    "4-star": (5, [(0, 1), (0, 2), (0, 3), (0, 4)]),
    "5-star": (6, [(0, 1), (0, 2), (0, 3), (0, 4), (0, 5)]),
    "6-star": (7, [(0, i) for i in range(1, 7)]),
    "5-path": (5, [(0, 1), (1, 2), (2, 3), (3, 4)]),
    "spider": (6, [(0, 1), (0, 2), (0, 3), (1, 4), (2, 5)]),
}

CONFIG_PATTERNS = {
    0: ["triangle", "4-cycle", "4-clique"],
    1: ["house", "5-cycle", "5-clique"],
    2: ["6-cycle", "6-cycle-chord", "prism", "k4-path", "5-wheel", "6-clique"],
    3: ["4-clique", "house", "5-cycle", "6-cycle-chord"],
}


def config_graph(idx: int) -> CSR:
    """The data graph of evaluation configuration ``idx`` (0..3)."""
    if idx == 0:
        return er(1000, 0.01, seed=1)
    if idx == 1:
        return rmat(17, 8, 0.57, 0.19, 0.19, seed=2)
    if idx == 2:
        return chung_lu(7000, 100_000, 2.1, seed=3)
    if idx == 3:
        return rmat(22, 8, 0.57, 0.19, 0.19, seed=4)
    raise ValueError(idx)


def random_connected_pattern(k: int, rng: np.random.Generator, p: float = 0.5):
    """A random connected pattern on k vertices (rejection sampling of G(k, p))."""
    pairs = list(itertools.combinations(range(k), 2))
    while True:
        edges = [e for e in pairs if rng.random() < p]
        adj = [set() for _ in range(k)]
        for a, b in edges:
            adj[a].add(b)
            adj[b].add(a)
        seen, stack = {0}, [0]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) == k:
            return edges


# ---------------------------------------------------------------- query streams

def connected_patterns(kmin: int = 3, kmax: int = 6) -> list:
    """One representative (k, edges) per isomorphism class of connected graphs
    on kmin..kmax vertices (2 + 6 + 21 + 112 = 141 classes for 3..6), in
    order of k, then of the canonical edge mask. The representative is the
    labelling whose edge mask (bit i = i-th pair of combinations(range(k), 2))
    is smallest in its class."""
    out = []
    for k in range(kmin, kmax + 1):
        pairs = list(itertools.combinations(range(k), 2))
        idx = {p: i for i, p in enumerate(pairs)}
        masks = np.arange(1 << len(pairs), dtype=np.int64)
        canon = masks.copy()
        for perm in itertools.permutations(range(k)):
            img = np.zeros_like(masks)
            for i, (a, b) in enumerate(pairs):
                t = idx[tuple(sorted((perm[a], perm[b])))]
                img |= ((masks >> i) & 1) << t
            np.minimum(canon, img, out=canon)
        for m in np.unique(canon):
            edges = [pairs[i] for i in range(len(pairs)) if (int(m) >> i) & 1]
            adj = [set() for _ in range(k)]
            for a, b in edges:
                adj[a].add(b)
                adj[b].add(a)
            seen, stack = {0}, [0]
            while stack:
                x = stack.pop()
                for y in adj[x]:
                    if y not in seen:
                        seen.add(y)
                        stack.append(y)
            if len(seen) == k:
                out.append((k, edges))
    return out


def poisson_stream(n: int = 2000, qps: float = 50.0, n_graphs: int = 3, n_patterns: int = 141,
                   seed: int = 5) -> list:
    """(arrival time in s, graph index, pattern index) for n queries with
    exponential inter-arrival times of mean 1/qps; graph and pattern drawn
    uniformly."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, n))
    gi = rng.integers(0, n_graphs, n)
    pi = rng.integers(0, n_patterns, n)
    return [(float(a), int(b), int(c)) for a, b, c in zip(t, gi, pi)]
