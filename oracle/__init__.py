"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU library
computes, written from the paper (GraphPi, arXiv 2009.10955). Only ``tests/``,
the smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it. It shares no code with the GPU library (``paper_2009_10955_amd``)
and imports nothing from it; graphs come in as any object with ``row_ptr``
(int64) and ``col`` (int32) arrays.

Contents and what each follows:

* ``count_maps`` / ``count`` / ``count_restricted`` -- the problem definition
  (Section II-A): injective maps sending every pattern edge onto a data edge;
  distinct subgraphs = maps / |Aut(P)| (Section II-B). Backtracking in C
  (``oracle.c``), 128-bit counts.
* ``brute_force_maps`` -- the same definition by exhaustive enumeration of all
  injective k-tuples, pure Python, tiny graphs only (pins the C oracle).
* ``automorphisms`` -- all vertex permutations that map the edge set onto
  itself (Section IV-A, Algorithm 1, first step).
* ``no_conflict``, ``validate``, ``restriction_sets`` -- Algorithm 1 (2-cycle
  based automorphism elimination), with the readings listed below.
* ``phase1_ok``, ``efficient_schedules`` -- the 2-phase schedule filter
  (Section IV-B).
* ``model_cost`` -- the nested performance model (Section IV-C).
* ``alg2_components``, ``alg2_cardinality``, ``iep_injective_tuples``,
  ``iep_count`` -- counting with the Inclusion-Exclusion Principle
  (Section IV-D, Algorithm 2).
* ``list_subgraphs`` -- the embeddings themselves (Section II-A: the problem
  is to find every subgraph that is an image of the pattern): each distinct
  subgraph once, as the set of its edges. Pure-Python backtracking, small
  graphs only.
* ``relabel_by_degree`` -- vertex relabelling by descending degree (ties by
  ascending id), the layout the GPU library uses; counts are invariant under it.

Readings of the paper used here (the paper is silent or garbled on these):

* Algorithm 1, 2-cycle test: a vertex v is on a 2-cycle of perm iff
  perm[perm[v]] == v and perm[v] != v (fixed points satisfy the first test too
  but are 1-cycles). The pair added is (v, perm[v]) (the listing's ``p`` is
  read as ``perm``).
* A pair (a, b) means id(a) > id(b), drawn as the directed edge a -> b.
* Closures: each restriction set is explored once per transitive closure.
  This is sound because whether a permutation conflicts with a set, and how
  many orders satisfy the set, depend only on its closure. A grown set's
  surviving automorphisms are its parent's survivors that do not conflict
  with it, the same as filtering all of Aut(P), since a permutation that
  conflicts with a set conflicts with every superset. The output is the list
  of distinct valid closures, sorted by size, then by their sorted pairs.
* ``validate`` runs the paper's check literally: count maps of the pattern into
  the complete graph K_k with and without the restrictions and require
  with * |Aut| == without.
* Phase 2 with no satisfying order: use the largest k' <= alpha(P) for which
  some Phase-1 order ends in k' pairwise non-adjacent vertices.
* IEP over-count: Section IV-D divides by the number of automorphisms that
  no_conflict does not eliminate with the remaining restrictions. That number
  is not the multiplicity in general (for K4 plus a pendant path with one kept
  restriction it is 5 while every embedding is counted 3 times, so the
  quotient is not even an integer). The division here uses the exact
  multiplicity: how many relative orders of each Aut-orbit obey the kept
  restrictions; a configuration for which that differs between orbits is not
  counted with IEP.
* Model: ``tri_cnt`` is the number of ordered triangles (6 x unordered), so
  ``tri_cnt / (2|E|)`` is the mean common-neighborhood size of an edge. A
  restriction is charged to the loop of its later-bound vertex. The loop of
  the i-th vertex has size |V| for i = 1, else the predicted size of the
  intersection of its parents' neighborhoods. An intersection is computed in
  the loop of its last-bound parent; it starts from the largest earlier
  candidate set whose parents are a subset of its own (computed in the same or
  an enclosing loop), else from the first parent's neighborhood, and
  intersects the remaining parents' neighborhoods in schedule order, each step
  costing the predicted sizes of both operands.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_count_maps.restype = ctypes.c_int
    lib.oracle_count_maps.argtypes = [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
        ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
        ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    _lib = lib
    return lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------- counting

def count_maps(g, k: int, edges: Sequence[tuple[int, int]], restr: Iterable[tuple[int, int]] = (),
               pins: Iterable[tuple[int, int]] = (), threads: int | None = None) -> int:
    """Number of injective maps id: V_p -> V_G with every pattern edge mapped to
    a data edge, id(a) > id(b) for every (a, b) in ``restr`` and id(u) = x for
    every (u, x) in ``pins``."""
    lib = _load()
    row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    n = row_ptr.shape[0] - 1
    e = _i32([x for ab in edges for x in ab])
    r = _i32([x for ab in restr for x in ab])
    pins = list(pins)
    pv = _i32([u for u, _ in pins])
    px = _i32([x for _, x in pins])
    lo = ctypes.c_uint64(0)
    hi = ctypes.c_uint64(0)
    rc = lib.oracle_count_maps(
        row_ptr.ctypes.data, col.ctypes.data, n, k, e.ctypes.data, len(edges),
        r.ctypes.data, r.size // 2, pv.ctypes.data, px.ctypes.data, len(pins),
        threads or default_threads(), ctypes.byref(lo), ctypes.byref(hi))
    if rc != 0:
        raise ValueError("oracle_count_maps: bad arguments")
    return (hi.value << 64) | lo.value


def automorphisms(k: int, edges: Sequence[tuple[int, int]]) -> list[tuple[int, ...]]:
    """All permutations p of 0..k-1 with {p(a), p(b)} an edge for every edge
    {a, b} (Section IV-A). p is returned as a tuple with p[v] = image of v."""
    es = {frozenset(e) for e in edges}
    out = []
    for p in itertools.permutations(range(k)):
        if all(frozenset((p[a], p[b])) in es for a, b in edges):
            out.append(p)
    return out


def count(g, k: int, edges, threads: int | None = None) -> int:
    """Number of distinct subgraphs of g isomorphic to (edge-preserving images
    of) the pattern: maps / |Aut(P)| (Section II-A/B)."""
    maps = count_maps(g, k, edges, threads=threads)
    aut = len(automorphisms(k, edges))
    if maps % aut:
        raise AssertionError("map count not divisible by |Aut|")
    return maps // aut


def count_restricted(g, k: int, edges, restr, threads: int | None = None) -> int:
    """Number of maps that satisfy every restriction pair (no division)."""
    return count_maps(g, k, edges, restr=restr, threads=threads)


def brute_force_maps(g, k: int, edges, restr=()) -> int:
    """Exhaustive count over all injective k-tuples (tiny graphs only)."""
    n = g.row_ptr.shape[0] - 1
    if n > 14:
        raise ValueError("brute_force_maps is for graphs with at most 14 vertices")
    adj = set()
    for v in range(n):
        for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
            adj.add((v, int(w)))
    total = 0
    for t in itertools.permutations(range(n), k):
        if all((t[a], t[b]) in adj for a, b in edges) and all(t[a] > t[b] for a, b in restr):
            total += 1
    return total


def list_subgraphs(g, k: int, edges) -> set:
    """Every distinct subgraph of g that is the image of an injective map
    sending each pattern edge onto a data edge (Section II-A), as a frozenset
    of its edges, each edge a (smaller id, larger id) pair. Two maps give the
    same subgraph exactly when they differ by an automorphism, so the result
    has maps / |Aut(P)| elements. Plain backtracking over pattern vertices
    0..k-1: a vertex with an earlier pattern neighbor ranges over the data
    neighbors of that neighbor's image, any other over all of V, and a
    partial map is dropped as soon as it repeats a vertex or misses a pattern
    edge to a bound vertex. Small graphs only."""
    row_ptr = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    nbr = [set(col[row_ptr[v]:row_ptr[v + 1]].tolist()) for v in range(n)]
    earlier = [[b for a, b in edges if a == u and b < u] + [a for a, b in edges if b == u and a < u]
               for u in range(k)]
    found = set()
    img = [0] * k

    def rec(u: int) -> None:
        if u == k:
            found.add(frozenset((min(img[a], img[b]), max(img[a], img[b])) for a, b in edges))
            return
        # a later vertex with an earlier pattern neighbor can only be one of
        # that neighbor's data neighbors; the rest range over all of V
        cands = sorted(nbr[img[earlier[u][0]]]) if earlier[u] else range(n)
        for x in cands:
            if x in img[:u]:
                continue
            if all(img[w] in nbr[x] for w in earlier[u]):
                img[u] = x
                rec(u + 1)

    rec(0)
    return found


def relabel_by_degree(g):
    """Relabel by descending degree, ties by ascending original id.
    Returns (row_ptr int64, col int32 with each list ascending, new_id)."""
    row_ptr = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    deg = np.diff(row_ptr)
    order = np.lexsort((np.arange(n), -deg))  # primary: -deg, secondary: id
    new_id = np.empty(n, dtype=np.int64)
    new_id[order] = np.arange(n)
    src = np.repeat(np.arange(n), deg)
    key = np.sort(new_id[src] * n + new_id[col])
    rows = key // n
    new_col = (key % n).astype(np.int32)
    new_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=new_ptr[1:])
    return new_ptr, new_col, new_id.astype(np.int32)


class _CSRView:
    def __init__(self, row_ptr, col):
        self.row_ptr = row_ptr
        self.col = col


def complete_graph(n: int):
    """K_n as CSR (used by ``validate``)."""
    rows = [[j for j in range(n) if j != i] for i in range(n)]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in r], dtype=np.int32)
    return _CSRView(row_ptr, col)


# ------------------------------------------------- Algorithm 1 (Section IV-A)

def closure(pairs: Iterable[tuple[int, int]], k: int) -> frozenset:
    """Transitive closure of the relation given by ``pairs``."""
    reach = [[False] * k for _ in range(k)]
    for a, b in pairs:
        reach[a][b] = True
    for m in range(k):
        for i in range(k):
            if reach[i][m]:
                for j in range(k):
                    if reach[m][j]:
                        reach[i][j] = True
    return frozenset((i, j) for i in range(k) for j in range(k) if reach[i][j])


def _acyclic(k: int, arcs: Iterable[tuple[int, int]]) -> bool:
    succ = [set() for _ in range(k)]
    indeg = [0] * k
    for a, b in set(arcs):
        if b not in succ[a]:
            succ[a].add(b)
            indeg[b] += 1
    ready = [v for v in range(k) if indeg[v] == 0]
    seen = 0
    while ready:
        v = ready.pop()
        seen += 1
        for w in succ[v]:
            indeg[w] -= 1
            if indeg[w] == 0:
                ready.append(w)
    return seen == k


def no_conflict(perm: Sequence[int], res_set: Iterable[tuple[int, int]]) -> bool:
    """Algorithm 1, no_conflict: put each restriction (a, b) and its image
    (perm[a], perm[b]) into a digraph; the permutation survives (is NOT
    eliminated) iff the digraph is acyclic."""
    k = len(perm)
    arcs = []
    for a, b in res_set:
        arcs.append((a, b))
        arcs.append((perm[a], perm[b]))
    return _acyclic(k, arcs)


def validate(k: int, edges, res_set, auts=None) -> bool:
    """Algorithm 1, validate: match the pattern on the complete graph K_k with
    and without the restrictions; valid iff with == without / |Aut|."""
    if auts is None:
        auts = automorphisms(k, edges)
    kk = complete_graph(k)
    without = count_maps(kk, k, edges, threads=1)
    with_r = count_maps(kk, k, edges, restr=sorted(res_set), threads=1)
    return with_r * len(auts) == without


def _two_cycle_pairs(perm: Sequence[int]) -> list[tuple[int, int]]:
    """(v, perm[v]) for every vertex v that perm swaps with another vertex."""
    return [(v, perm[v]) for v in range(len(perm)) if perm[v] != v and perm[perm[v]] == v]


def restriction_sets(k: int, edges, max_states: int | None = None) -> list[frozenset]:
    """Section IV-A (Algorithm 1): restriction sets that eliminate every
    automorphism but the identity.

    Starting from the empty set, a set R grows by one pair (v, perm[v]) at a
    time, where perm is an automorphism that R has not yet eliminated
    (no_conflict(perm, R) holds) and v lies on a 2-cycle of perm. A set at
    which the identity alone survives is a candidate, kept if validate
    accepts it. Sets are handled as their transitive closures (reading in the
    module header), the reachable closures are explored once each from a
    worklist, and the distinct valid closures are returned sorted by size and
    then by their sorted pairs (the paper fixes no order)."""
    auts = automorphisms(k, edges)
    start = frozenset()
    seen = {start}
    # (closure, the automorphisms it has not eliminated); a grown closure
    # keeps those of its parent's survivors that do not conflict with it,
    # the same as filtering all of Aut(P) since conflicts persist in supersets
    work = [(start, auts)]
    valid: set = set()
    while work:
        rel, alive = work.pop()
        if len(alive) <= 1:
            # the identity alone survives (or nothing does: a cyclic set)
            if alive and validate(k, edges, rel, auts):
                valid.add(rel)
            continue
        for perm in alive:
            for pair in _two_cycle_pairs(perm):
                grown = closure(rel | {pair}, k)
                if grown in seen:
                    continue
                if max_states is not None and len(seen) >= max_states:
                    continue
                seen.add(grown)
                work.append((grown, [p for p in alive if no_conflict(p, grown)]))
    return sorted(valid, key=lambda r: (len(r), sorted(r)))


# --------------------------------------------- schedules (Section IV-B)

def _adj(k: int, edges):
    adj = [[False] * k for _ in range(k)]
    for a, b in edges:
        adj[a][b] = adj[b][a] = True
    return adj


def phase1_ok(order: Sequence[int], adj) -> bool:
    """Every searched vertex after the first is adjacent to an earlier one."""
    return all(any(adj[order[i]][order[j]] for j in range(i)) for i in range(1, len(order)))


def independence_number(k: int, adj) -> int:
    best = 0
    for r in range(1, k + 1):
        for s in itertools.combinations(range(k), r):
            if all(not adj[a][b] for a, b in itertools.combinations(s, 2)):
                best = r
                break
    return best


def efficient_schedules(k: int, edges) -> tuple[list[tuple[int, ...]], int]:
    """Phase 1 then Phase 2. Returns (schedules, k_eff)."""
    adj = _adj(k, edges)
    p1 = [o for o in itertools.permutations(range(k)) if phase1_ok(o, adj)]
    alpha = independence_number(k, adj)
    for keff in range(alpha, 0, -1):
        sel = [o for o in p1
               if all(not adj[a][b] for a, b in itertools.combinations(o[k - keff:], 2))]
        if sel:
            return sel, keff
    return p1, 0


# ------------------------------------- performance model (Section IV-C)

def predicted_card(nsets: int, n_v: float, n_e: float, tri_cnt: float) -> float:
    """Predicted size of the intersection of ``nsets`` neighborhoods:
    |V| p1 p2^(nsets-1), p1 = 2|E|/|V|^2, p2 = tri_cnt |V| / (2|E|)^2."""
    p1 = 2.0 * n_e / (n_v * n_v)
    p2 = tri_cnt * n_v / ((2.0 * n_e) ** 2)
    return n_v * p1 * p2 ** (nsets - 1)


def filter_fractions(k: int, order: Sequence[int], res_set) -> list[float]:
    """f for each loop: start from all k! relative magnitudes and, loop by loop,
    drop those violating the restrictions checked in that loop (a restriction
    is checked in the loop of its later-bound vertex); f is the fraction of the
    loop's incoming survivors that is dropped."""
    pos = {u: i for i, u in enumerate(order)}
    survivors = list(itertools.permutations(range(k)))
    f = [0.0] * k
    for i in range(k):
        here = [(a, b) for a, b in res_set if max(pos[a], pos[b]) == i]
        if not here:
            continue
        before = len(survivors)
        survivors = [r for r in survivors if all(r[a] > r[b] for a, b in here)]
        f[i] = (before - len(survivors)) / before if before else 0.0
    return f


def model_cost(k: int, edges, order: Sequence[int], res_set, n_v: float, n_e: float,
               tri_cnt: float) -> float:
    """cost_1 of the nested model for schedule ``order`` and restriction set
    ``res_set`` (pairs over pattern vertices), with graph stats |V|, |E|
    (undirected) and tri_cnt (ordered triangles):
    cost_i = l_i (1 - f_i) (c_i + cost_{i+1}),  cost_n = l_n (1 - f_n)."""
    adj = _adj(k, edges)

    def card(nsets: int) -> float:
        return predicted_card(nsets, n_v, n_e, tri_cnt)

    parents = [[j for j in range(i) if adj[order[i]][order[j]]] for i in range(k)]
    f = filter_fractions(k, order, res_set)

    # loop sizes
    loop = [0.0] * k
    loop[0] = n_v
    for i in range(1, k):
        loop[i] = card(len(parents[i]))

    # intersection costs, charged to the loop of the last-bound parent
    c = [0.0] * k
    built: list[int] = []   # levels whose candidate set is an intersection
    for i in range(k):
        ps = parents[i]
        if len(ps) < 2:
            continue
        h = max(ps)
        base = None
        for m in built:
            pm = parents[m]
            if max(pm) <= h and set(pm) < set(ps):
                if base is None or len(pm) > len(parents[base]):
                    base = m
        if base is None:
            have = 1
            rest = ps[1:]
        else:
            have = len(parents[base])
            rest = [j for j in ps if j not in parents[base]]
        for _ in rest:
            c[h] += card(have) + card(1)
            have += 1
        built.append(i)

    cost = loop[k - 1] * (1.0 - f[k - 1])
    for i in range(k - 2, -1, -1):
        cost = loop[i] * (1.0 - f[i]) * (c[i] + cost)
    return cost


# ------------------------------------- inclusion-exclusion counting (Section IV-D)

def alg2_components(k: int, pairs) -> list[list[int]]:
    """Algorithm 2, lines 1-4: the undirected graph on k set indices with one
    edge per (i, j) pair, split into connected components (each sorted)."""
    parent = list(range(k))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    comps: dict = {}
    for v in range(k):
        comps.setdefault(find(v), []).append(v)
    return sorted(sorted(c) for c in comps.values())


def alg2_cardinality(sets, pairs) -> int:
    """Algorithm 2: |A_{i1,j1} ∩ ... ∩ A_{im,jm}| = product over the components
    of the pair graph of the size of the intersection of their sets."""
    card = 1
    for comp in alg2_components(len(sets), pairs):
        inter = set(sets[comp[0]])
        for v in comp[1:]:
            inter &= set(sets[v])
        card *= len(inter)
    return card


def iep_injective_tuples(sets) -> int:
    """|S_IEP|: tuples (e_1..e_k), e_i in S_i, all distinct, by the
    inclusion-exclusion sum over subsets of the pairs (i<j) of
    (-1)^|subset| |∩ A_{i,j}| (Section IV-D), each term by Algorithm 2."""
    k = len(sets)
    pairs = list(itertools.combinations(range(k), 2))
    total = 0
    for r in range(len(pairs) + 1):
        for sub in itertools.combinations(pairs, r):
            total += (-1) ** r * alg2_cardinality(sets, sub)
    return total


def iep_kept(k: int, order, res_set, n_inner: int) -> list:
    """The restrictions that remain with IEP: those checked in the outer
    loops (the later-bound vertex is not among the last n_inner)."""
    pos = {u: i for i, u in enumerate(order)}
    return [(a, b) for a, b in res_set if max(pos[a], pos[b]) < k - n_inner]


def iep_divisor_paper(k: int, edges, order, res_set, n_inner: int) -> int:
    """x as Section IV-D computes it: the automorphisms that no_conflict does
    not eliminate with the remaining restrictions."""
    kept = iep_kept(k, order, res_set, n_inner)
    return sum(1 for p in automorphisms(k, edges) if no_conflict(p, kept))


def orbit_multiplicities(k: int, edges, kept) -> set:
    """For every Aut-orbit of the k! relative orders, how many of its members
    obey all pairs in kept. IEP over-counts each embedding by exactly this
    number, so it is usable only when the set has one element."""
    auts = automorphisms(k, edges)
    seen: set = set()
    out: set = set()
    for r in itertools.permutations(range(k)):
        orbit = frozenset(tuple(r[p[v]] for v in range(k)) for p in auts)
        if orbit in seen:
            continue
        seen.add(orbit)
        out.add(sum(all(x[a] > x[b] for a, b in kept) for x in orbit))
    return out


def iep_divisor(k: int, edges, order, res_set, n_inner: int) -> int:
    """The exact over-count of IEP counting: the number of relative orders in
    each Aut-orbit that obey the remaining restrictions (every maps' orbit of
    one embedding has this many members counted). Raises if it is not the
    same for every orbit, which happens for some configurations (then IEP
    does not apply to them). Section IV-D's no_conflict count
    (iep_divisor_paper) equals it only in some cases."""
    m = orbit_multiplicities(k, edges, iep_kept(k, order, res_set, n_inner))
    if len(m) != 1:
        raise ValueError(f"IEP over-count is not uniform over orbits: {sorted(m)}")
    return m.pop()


def iep_count(g, k: int, edges, order, res_set, n_inner: int) -> int:
    """Embeddings counted the IEP way of Section IV-D (small graphs only):
    enumerate the outer k - n_inner vertices of the schedule under the
    restrictions checked in those loops, take for each inner vertex its
    candidate set (the common neighbors of its pattern neighbors' images,
    minus the outer images), count the distinct-entry tuples by
    inclusion-exclusion, and divide the total by the over-count (the exact
    per-orbit multiplicity, see iep_divisor)."""
    adj = _adj(k, edges)
    inner = list(order[k - n_inner:])
    outer = list(order[:k - n_inner])
    for a, b in itertools.combinations(inner, 2):
        if adj[a][b]:
            raise ValueError("inner vertices must be pairwise non-adjacent")
    kept = iep_kept(k, order, res_set, n_inner)
    x = iep_divisor(k, edges, order, res_set, n_inner)
    n = g.row_ptr.shape[0] - 1
    nbr = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(n)]
    total = 0
    img: dict = {}

    def rec(t):
        nonlocal total
        if t == len(outer):
            used = set(img.values())
            sets = []
            for u in inner:
                cand = None
                for w in range(k):
                    if adj[u][w]:
                        s = nbr[img[w]]
                        cand = set(s) if cand is None else cand & s
                cand = (cand if cand is not None else set(range(n))) - used
                sets.append(cand)
            total += iep_injective_tuples(sets)
            return
        u = outer[t]
        for x in range(n):
            if x in img.values():
                continue
            if any(adj[u][w] and w in img and x not in nbr[img[w]] for w in range(k)):
                continue
            img[u] = x
            if all(img[a] > img[b] for a, b in kept if a in img and b in img):
                rec(t + 1)
            del img[u]

    rec(0)
    if total % x:
        raise AssertionError("IEP total not divisible by x")
    return total // x
