"""Pins for the CPU oracle: each test checks it against something other than
itself -- exhaustive enumeration, textbook closed forms, library routines,
invariants, and the values the paper prints for its worked examples."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2009_10955_amd import inputs as I

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))
P = I.PATTERNS


def _graph_from_mask(n, mask):
    pairs = list(itertools.combinations(range(n), 2))
    src = [a for t, (a, b) in enumerate(pairs) if mask >> t & 1]
    dst = [b for t, (a, b) in enumerate(pairs) if mask >> t & 1]
    return I.csr_from_edges(n, np.array(src, dtype=np.int64), np.array(dst, dtype=np.int64))


# ------------------------------------------------ C oracle vs exhaustive search

@pytest.mark.parametrize("pname", ["edge", "triangle", "4-path", "3-star", "4-cycle",
                                   "tailed-triangle", "diamond", "4-clique"])
def test_maps_match_exhaustive_on_all_5_vertex_graphs(pname):
    """Every graph on 5 labelled vertices (all 2^10 edge subsets)."""
    k, e = P[pname]
    for mask in range(1 << 10):
        g = _graph_from_mask(5, mask)
        assert O.count_maps(g, k, e, threads=1) == O.brute_force_maps(g, k, e), (pname, mask)


@pytest.mark.parametrize("seed", [11, 12, 13])
@pytest.mark.parametrize("pname", ["house", "5-cycle", "5-clique", "4-cycle", "diamond"])
def test_maps_match_exhaustive_on_random_graphs(seed, pname):
    k, e = P[pname]
    g = I.er(10, 0.55, seed=seed)
    assert O.count_maps(g, k, e) == O.brute_force_maps(g, k, e)


@pytest.mark.parametrize("seed", [21, 22])
def test_restricted_and_pinned_maps_match_exhaustive(seed):
    """Restriction pairs and pinned vertices, checked by enumeration."""
    g = I.er(9, 0.6, seed=seed)
    k, e = P["house"]
    restr = [(0, 1), (3, 2)]
    assert O.count_maps(g, k, e, restr=restr) == O.brute_force_maps(g, k, e, restr)
    # pins split the count exactly: sum over the image of vertex 0 and 1
    total = 0
    for a in range(g.n):
        for b in g.neighbors(a):
            total += O.count_maps(g, k, e, restr=restr, pins=[(0, a), (1, int(b))])
    assert total == O.count_maps(g, k, e, restr=restr)


def test_six_vertex_patterns_match_exhaustive():
    g = I.er(9, 0.7, seed=5)
    for pname in ["6-cycle", "prism", "5-wheel", "6-cycle-chord"]:
        k, e = P[pname]
        assert O.count_maps(g, k, e) == O.brute_force_maps(g, k, e), pname


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("pname", list(P))
def test_complete_graph_closed_form(pname):
    """In K_n every injective map is edge-preserving: maps = n!/(n-k)!, and
    subgraphs = C(n, k) k! / |Aut(P)|."""
    k, e = P[pname]
    n = 8
    aut = len(O.automorphisms(k, e))
    assert O.count(I.complete(n), k, e) == math.comb(n, k) * math.factorial(k) // aut


def test_complete_bipartite_closed_forms():
    for a, b in [(3, 4), (5, 5), (2, 7)]:
        g = I.complete_bipartite(a, b)
        assert O.count(g, *P["4-cycle"]) == math.comb(a, 2) * math.comb(b, 2)
        assert O.count(g, *P["triangle"]) == 0
        assert O.count(g, *P["5-cycle"]) == 0  # bipartite: no odd cycles


@pytest.mark.parametrize("d", [3, 4, 5])
def test_hypercube_four_cycles(d):
    assert O.count(I.hypercube(d), *P["4-cycle"]) == math.comb(d, 2) * 2 ** (d - 2)


@pytest.mark.parametrize("m", [5, 6, 9])
def test_cycle_graph_has_one_m_cycle(m):
    g = I.cycle_graph(m)
    cyc = (m, [(i, (i + 1) % m) for i in range(m)])
    assert O.count(g, *cyc) == 1
    assert O.count(g, *P["triangle"]) == 0


def test_star_counts_are_degree_binomials():
    g = I.er(60, 0.2, seed=7)
    deg = g.degrees()
    assert O.count(g, *P["3-star"]) == sum(math.comb(int(d), 3) for d in deg)
    assert O.count(g, *P["edge"]) == g.m
    assert O.count(I.star(7), *P["3-star"]) == math.comb(7, 3)


def test_trace_formulas():
    """triangles = tr(A^3)/6 ; 4-cycles = (tr(A^4) - 2 sum d^2 + 2m) / 8."""
    g = I.er(40, 0.2, seed=3)
    A = np.zeros((g.n, g.n), dtype=np.int64)
    for v in range(g.n):
        A[v, g.neighbors(v)] = 1
    A2 = A @ A
    deg = A.sum(1)
    tri = int(np.trace(A2 @ A)) // 6
    c4 = (int(np.trace(A2 @ A2)) - 2 * int((deg ** 2).sum()) + 2 * g.m) // 8
    assert O.count(g, *P["triangle"]) == tri
    assert O.count(g, *P["4-cycle"]) == c4


@pytest.mark.parametrize("cfg", [0, 2])
def test_triangles_match_scipy_on_config_graphs(cfg):
    g = I.config_graph(cfg)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    tri = int(round((A @ A).multiply(A).sum() / 6))
    assert O.count(g, *P["triangle"]) == tri


def test_disjoint_union_adds_and_relabel_preserves():
    g = I.er(30, 0.3, seed=8)
    h = I.er(25, 0.35, seed=9)
    u = I.disjoint_union(g, h)
    rng = np.random.default_rng(0)
    perm = rng.permutation(u.n)
    pu = I.permute(u, perm)
    for pname in ["triangle", "4-cycle", "house", "diamond"]:
        k, e = P[pname]
        cg, ch = O.count(g, k, e), O.count(h, k, e)
        assert O.count(u, k, e) == cg + ch
        assert O.count(pu, k, e) == cg + ch


def test_relabel_by_degree():
    g = I.config_graph(2)
    rp, col, new_id = O.relabel_by_degree(g)
    deg_new = np.diff(rp)
    assert np.all(deg_new[:-1] >= deg_new[1:])                  # descending degree
    assert sorted(new_id.tolist()) == list(range(g.n))           # a permutation
    # ties keep ascending original id
    old_of_new = np.argsort(new_id)
    same = deg_new[:-1] == deg_new[1:]
    assert np.all(old_of_new[:-1][same] < old_of_new[1:][same])
    for v in range(0, g.n, 97):                                  # same edges
        nb = sorted(new_id[g.neighbors(v)].tolist())
        w = new_id[v]
        assert col[rp[w]:rp[w + 1]].tolist() == nb


# ------------------------------------------------------------ automorphisms

def test_clique7_automorphisms_paper_value():
    gd = GOLDEN["clique7_automorphisms"]
    k = gd["k"]
    e = list(itertools.combinations(range(k), 2))
    assert len(O.automorphisms(k, e)) == gd["value"]


def test_automorphism_textbook_values():
    # cycles: dihedral group of order 2k; cliques: k!; stars K_{1,s}: s!
    for k in range(3, 8):
        assert len(O.automorphisms(k, [(i, (i + 1) % k) for i in range(k)])) == 2 * k
        assert len(O.automorphisms(k, list(itertools.combinations(range(k), 2)))) == math.factorial(k)
        assert len(O.automorphisms(k, [(0, i) for i in range(1, k)])) == math.factorial(k - 1)
    # paths: 2; prism (= C3 x K2): 12; wheel W5 (hub + 5-cycle): 10
    assert len(O.automorphisms(5, [(i, i + 1) for i in range(4)])) == 2
    assert len(O.automorphisms(*P["prism"])) == 12
    assert len(O.automorphisms(*P["5-wheel"])) == 10


# ---------------------------------------------------------- Algorithm 1

def test_rectangle_worked_example():
    gd = GOLDEN["rectangle_round1"]
    k, e = gd["k"], [tuple(x) for x in gd["edges"]]
    auts = O.automorphisms(k, e)
    assert tuple(gd["automorphism_swap_B_D"]) in auts
    r1 = [tuple(x) for x in gd["round1_set"]]
    rot = tuple(gd["rotation_eliminated"])
    assert rot in auts
    assert not O.no_conflict(rot, r1)            # the rotation is eliminated
    assert O.no_conflict(tuple(range(k)), r1)    # the identity never is
    survivors = [p for p in auts if O.no_conflict(p, r1)]
    # after round 1 exactly the identity and (A B)(C D) remain, so round 1 is
    # not the end: Fig. permutation_group (d) needs another round
    assert sorted(survivors) == sorted([(0, 1, 2, 3), (1, 0, 3, 2)])
    sets = O.restriction_sets(k, e)
    assert any(set(r1) <= s for s in sets)


def _linear_extensions(k, res):
    return sum(1 for r in itertools.permutations(range(k)) if all(r[a] > r[b] for a, b in res))


@pytest.mark.parametrize("pname", ["triangle", "4-cycle", "4-clique", "house", "5-cycle",
                                   "diamond", "tailed-triangle", "4-path", "3-star",
                                   "6-cycle-chord", "k4-path"])
def test_every_emitted_set_breaks_every_symmetry_exactly_once(pname):
    """For every emitted set: each Aut-orbit of the k! relative orders has
    exactly one member obeying it (so k!/|Aut| orders obey it), and on real
    graphs restricted maps * |Aut| == all maps."""
    k, e = P[pname]
    auts = O.automorphisms(k, e)
    sets = O.restriction_sets(k, e)
    assert sets
    g = I.er(11, 0.55, seed=4)
    g0 = I.config_graph(0)
    all_maps = O.count_maps(g, k, e)
    all_maps0 = O.count_maps(g0, k, e)
    for s in sets:
        assert _linear_extensions(k, s) * len(auts) == math.factorial(k)
        seen = set()
        for r in itertools.permutations(range(k)):
            orbit = frozenset(tuple(r[p[v]] for v in range(k)) for p in auts)
            if orbit in seen:
                continue
            seen.add(orbit)
            assert sum(all(x[a] > x[b] for a, b in s) for x in orbit) == 1
        assert O.count_maps(g, k, e, restr=s) * len(auts) == all_maps
        assert O.count_maps(g0, k, e, restr=s) * len(auts) == all_maps0


def test_count_restricted_equals_the_subgraph_count():
    """count_restricted (maps obeying a restriction set, no division) is the
    subgraph count for every emitted set, on a graph checked exhaustively
    elsewhere; brute force over all injective tuples agrees."""
    g = I.er(9, 0.6, seed=12)
    for pname in ["house", "5-cycle", "tailed-triangle"]:
        k, e = P[pname]
        want = O.count(g, k, e)
        for s in O.restriction_sets(k, e):
            assert O.count_restricted(g, k, e, s) == want
            assert O.brute_force_maps(g, k, e, s) == want


# independence numbers worked out by hand from the edge lists (a largest set
# of pairwise non-adjacent pattern vertices is named for each)
ALPHA = {"edge": 1, "triangle": 1, "4-clique": 1, "5-clique": 1, "6-clique": 1,
         "4-cycle": 2,          # {0, 2}
         "house": 2,            # {2, 4}
         "5-cycle": 2,          # {0, 2}
         "6-cycle": 3,          # {0, 2, 4}
         "6-cycle-chord": 3,    # {1, 3, 5}
         "prism": 2,            # one vertex per triangle, not matched
         "k4-path": 2,          # {0, 4}: one K4 vertex, one of 4, 5
         "5-wheel": 2,          # two of the rim
         "4-path": 2, "5-path": 3,  # alternate vertices of the path
         "3-star": 3, "4-star": 4, "5-star": 5, "6-star": 6,  # the leaves
         "tailed-triangle": 2,  # {0, 3}
         "diamond": 2,          # {1, 3}
         "spider": 3}           # {3, 4, 5}


@pytest.mark.parametrize("pname", sorted(ALPHA))
def test_independence_number_hand_values(pname):
    """The bound on the inner loops that Phase 2 and IEP use (Section IV-B,
    IV-D): the largest independent set of the pattern, and no schedule ends
    in more independent vertices than it."""
    k, e = P[pname]
    assert O.independence_number(k, O._adj(k, e)) == ALPHA[pname]
    _, keff = O.efficient_schedules(k, e)
    assert 1 <= keff <= ALPHA[pname]


def test_iep_kept_drops_restrictions_on_the_inner_loops():
    """With the last n_inner schedule vertices counted by inclusion-exclusion,
    only the restrictions between outer vertices are still checked."""
    res = [(1, 0), (4, 2), (3, 0), (2, 1)]
    assert O.iep_kept(5, (0, 1, 2, 3, 4), res, 2) == [(1, 0), (2, 1)]
    assert O.iep_kept(5, (4, 3, 2, 1, 0), res, 2) == [(4, 2)]
    assert O.iep_kept(5, (0, 1, 2, 3, 4), res, 0) == res


def test_invalid_set_is_rejected_by_validate():
    k, e = P["4-cycle"]
    assert not O.validate(k, e, [(0, 1)])                  # too few restrictions
    assert not O.validate(k, e, [(0, 1), (1, 2), (2, 3), (0, 2), (0, 3), (1, 3)])  # too many
    assert O.validate(k, e, O.closure([(0, 1), (0, 2), (0, 3), (1, 3)], k))


# ------------------------------------------------------------ schedules

def test_house_schedule_example():
    gd = GOLDEN["house_schedule"]
    k, e = gd["k"], [tuple(x) for x in gd["edges"]]
    scheds, keff = O.efficient_schedules(k, e)
    assert keff == gd["phase2_k"]
    assert tuple(gd["efficient_schedule"]) in scheds
    adj = O._adj(k, e)
    bad = gd["phase1_violating_prefix"]
    rest = [u for u in range(k) if u not in bad]
    for tail in itertools.permutations(rest):
        assert not O.phase1_ok(list(bad) + list(tail), adj)


def test_schedules_are_prefix_connected_and_end_independent():
    for pname in ["house", "prism", "5-wheel", "6-cycle-chord", "k4-path", "6-cycle"]:
        k, e = P[pname]
        adj = O._adj(k, e)
        scheds, keff = O.efficient_schedules(k, e)
        assert scheds
        for o in scheds:
            for i in range(1, k):   # first i vertices induce a connected graph
                seen, stack = {o[0]}, [o[0]]
                while stack:
                    x = stack.pop()
                    for y in o[:i + 1]:
                        if adj[x][y] and y not in seen:
                            seen.add(y)
                            stack.append(y)
                assert len(seen) == i + 1
            tail = o[k - keff:]
            assert all(not adj[a][b] for a, b in itertools.combinations(tail, 2))


# ------------------------------------------------------------------ model

def test_filter_fraction_example():
    gd = GOLDEN["house_filter_fraction"]
    f = O.filter_fractions(gd["k"], list(range(gd["k"])), [tuple(x) for x in gd["restriction"]])
    assert f[1] == gd["f"]          # charged to the loop of B, the later-bound vertex
    assert sum(f) == gd["f"]


def test_cardinality_forms():
    g = I.config_graph(2)
    n_v, n_e = g.n, g.m
    tri = 6 * O.count(g, *P["triangle"])
    assert math.isclose(O.predicted_card(1, n_v, n_e, tri), 2 * n_e / n_v)
    assert math.isclose(O.predicted_card(2, n_v, n_e, tri), tri / (2 * n_e))
    # tri/(2|E|) is the exact mean common-neighborhood size over directed edges
    common = 0
    for v in range(g.n):
        nv = set(g.neighbors(v).tolist())
        for w in g.neighbors(v):
            common += len(nv & set(g.neighbors(int(w)).tolist()))
    assert math.isclose(O.predicted_card(2, n_v, n_e, tri), common / (2 * n_e))


def test_model_without_intersections_or_filters_is_product_of_loops():
    k, e = P["3-star"]
    n_v, n_e, tri = 1000.0, 5000.0, 900.0
    cost = O.model_cost(k, e, (0, 1, 2, 3), [], n_v, n_e, tri)
    assert math.isclose(cost, n_v * (2 * n_e / n_v) ** 3)


def test_model_prefers_hoisted_intersections_and_filters():
    """A schedule whose intersection sits in an outer loop costs less than one
    that recomputes it in an inner loop; more early filtering costs less."""
    k, e = P["house"]
    n_v, n_e, tri = 1e5, 1e6, 6e6
    # E (4) intersects N(A) and N(B): computed in loop 2 for (0,1,4,...) order
    hoisted = O.model_cost(k, e, (0, 1, 4, 3, 2), [], n_v, n_e, tri)
    inner = O.model_cost(k, e, (0, 3, 2, 1, 4), [], n_v, n_e, tri)
    assert hoisted < inner
    a = O.model_cost(k, e, (0, 1, 2, 3, 4), [(0, 1)], n_v, n_e, tri)
    b = O.model_cost(k, e, (0, 1, 2, 3, 4), [], n_v, n_e, tri)
    assert a < b


# Hand-derived values of cost_1 (Section IV-C) on |V| = 1000, |E| = 5000,
# tri_cnt = 6000 (ordered triangles). With d = 2|E|/|V| = 10 (one
# neighborhood) and q = |V| p1 p2 = tri_cnt / (2|E|) = 0.6 (two), p2 = 0.06.
#
# House of Fig. pseudocode_performance: schedule A,B,C,D,E = 0..4, the one
# restriction id(A) > id(B), charged to B's loop (f_2 = 1/2). Loops:
#   A: l = 1000, f = 0, c = 0
#   B: l = d, f = 1/2, c = |N(A)| + |N(B)| = 2d   (tmp_AB = N(A) & N(B), E's set)
#   C: l = d, f = 0, c = |N(A)| + |N(C)| = 2d     (N(A) & N(C), D's set)
#   D: l = q;  E: l = q
#   cost_5 = q; cost_4 = q * q; cost_3 = d (2d + q^2) = 203.6
#   cost_2 = d (1/2) (2d + cost_3) = 5 * 223.6 = 1118; cost_1 = 1000 * 1118
HOUSE_COST = 1_118_000.0
# 4-clique, schedule 0,1,2,3, restrictions 0 > 1 > 2 > 3 (closure):
#   f_2 = 1/2 (0>1), f_3 = 2/3 (12 orders left, 4 keep 0>1>2), f_4 = 3/4
#   level 2's set N(0) & N(1) costs 2d in loop 2; level 3's set extends it
#   by N(2) in loop 3: c_3 = q + d = 10.6 (the earlier set is the base)
#   l_4 = |V| p1 p2^2 = 0.036: cost_4 = 0.036 / 4 = 0.009
#   cost_3 = q (1/3) (10.6 + 0.009) = 2.1218; cost_2 = d (1/2) (2d + 2.1218) = 110.609
#   cost_1 = 1000 * 110.609
CLIQUE4_COST = 110_609.0


def test_model_hand_derived_values():
    """cost_1 literals worked out by hand from Section IV-C's definitions
    (above): a dropped term, a restriction charged to the wrong loop, an
    intersection charged to the wrong loop or built from the wrong base all
    change them."""
    k, e = P["house"]
    got = O.model_cost(k, e, (0, 1, 2, 3, 4), {(0, 1)}, 1000.0, 5000.0, 6000.0)
    assert math.isclose(got, HOUSE_COST, rel_tol=1e-12)
    k, e = P["4-clique"]
    r = O.closure([(0, 1), (1, 2), (2, 3)], 4)
    got = O.model_cost(k, e, (0, 1, 2, 3), r, 1000.0, 5000.0, 6000.0)
    assert math.isclose(got, CLIQUE4_COST, rel_tol=1e-12)
    assert O.filter_fractions(4, (0, 1, 2, 3), r) == [0.0, 0.5, 2.0 / 3.0, 0.75]


# ------------------------------------------------------- IEP (Section IV-D)

def test_alg2_worked_example():
    gd = GOLDEN["alg2_components"]
    pairs = [(a - 1, b - 1) for a, b in gd["pairs"]]
    comps = O.alg2_components(gd["k"], pairs)
    assert [[v + 1 for v in c] for c in comps] == gd["components"]
    sets = [{1, 2, 3}, {2, 3, 4}, {3, 4}, {5, 6, 7}, {6, 7}, {8, 9}]
    # |S1 ∩ S2 ∩ S3| * |S4 ∩ S5| * |S6|
    assert O.alg2_cardinality(sets, pairs) == 1 * 2 * 2


@pytest.mark.parametrize("seed", range(6))
def test_iep_sum_counts_distinct_tuples(seed):
    rng = np.random.default_rng(seed)
    for k in (1, 2, 3, 4):
        sets = [set(rng.choice(9, size=int(rng.integers(0, 7)), replace=False).tolist())
                for _ in range(k)]
        brute = sum(1 for t in itertools.product(*[sorted(s) for s in sets]) if len(set(t)) == k)
        assert O.iep_injective_tuples(sets) == brute


@pytest.mark.parametrize("pname", ["house", "diamond", "tailed-triangle", "4-path", "3-star",
                                   "6-cycle-chord", "k4-path"])
def test_iep_count_equals_plain_count(pname):
    """Every configuration with a uniform over-count gives the plain count."""
    k, e = P[pname]
    g = I.er(13, 0.45, seed=3)
    want = O.count(g, k, e)
    scheds, keff = O.efficient_schedules(k, e)
    sets = O.restriction_sets(k, e)
    n_ok = 0
    for o in scheds[:5]:
        for r in sets[:6]:
            for ni in range(2, keff + 1):
                try:
                    O.iep_divisor(k, e, o, r, ni)
                except ValueError:
                    continue
                assert O.iep_count(g, k, e, o, r, ni) == want, (o, sorted(r), ni)
                n_ok += 1
    assert n_ok > 0


def test_iep_paper_divisor_differs_from_the_multiplicity():
    """K4 plus a pendant path, schedule (0,1,3,4,2,5), set {0>1, 0>2, 1>2}:
    the only restriction checked outside the last two loops is 0>1. Every
    embedding is then counted 3 times (half of the 6 orders of K4's
    vertices 0,1,2 obey 0>1), but no_conflict leaves 5 automorphisms."""
    k, e = P["k4-path"]
    order = (0, 1, 3, 4, 2, 5)
    r = [(0, 1), (0, 2), (1, 2)]
    assert O.iep_divisor_paper(k, e, order, r, 2) == 5
    assert O.iep_divisor(k, e, order, r, 2) == 3
    g = I.er(12, 0.5, seed=4)
    assert O.iep_count(g, k, e, order, r, 2) == O.count(g, k, e)


# ------------------------------------------------------------ listing (II-A)

def _edge_sets_by_permutations(g, k, edges):
    """Image edge sets of every injective k-tuple that maps each pattern edge
    onto a data edge, by exhaustive enumeration of tuples (tiny graphs)."""
    n = g.row_ptr.shape[0] - 1
    adj = {(v, int(w)) for v in range(n) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]}
    out = set()
    for t in itertools.permutations(range(n), k):
        if all((t[a], t[b]) in adj for a, b in edges):
            out.add(frozenset((min(t[a], t[b]), max(t[a], t[b])) for a, b in edges))
    return out


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_listing_cliques_of_complete_graph(k):
    """K_6: the k-cliques are the C(6, k) vertex subsets, each with all its pairs."""
    edges = list(itertools.combinations(range(k), 2))
    got = O.list_subgraphs(I.complete(6), k, edges)
    want = {frozenset(itertools.combinations(s, 2)) for s in itertools.combinations(range(6), k)}
    assert got == want and len(got) == math.comb(6, k)


def test_listing_four_cycles_of_k4_and_wedges_of_a_star():
    """K_4 holds exactly its 3 Hamiltonian cycles; a star with s leaves holds
    C(s, 2) wedges, each two spokes."""
    c4 = O.list_subgraphs(I.complete(4), 4, P["4-cycle"][1])
    assert c4 == {frozenset({(0, 1), (1, 2), (2, 3), (0, 3)}), frozenset({(0, 1), (1, 3), (2, 3), (0, 2)}),
                  frozenset({(0, 2), (1, 2), (1, 3), (0, 3)})}
    s = 7
    wedges = O.list_subgraphs(I.star(s), 3, [(0, 1), (1, 2)])
    assert wedges == {frozenset({(0, i), (0, j)}) for i, j in itertools.combinations(range(1, s + 1), 2)}


@pytest.mark.parametrize("m", [4, 5, 6])
def test_listing_cycle_graph_is_itself(m):
    g = I.cycle_graph(m)
    edges = [(i, (i + 1) % m) for i in range(m)]
    got = O.list_subgraphs(g, m, edges)
    assert got == {frozenset((min(i, (i + 1) % m), max(i, (i + 1) % m)) for i in range(m))}


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("pname", ["triangle", "4-cycle", "diamond", "house", "5-cycle", "tailed-triangle"])
def test_listing_matches_exhaustive_tuples_and_count(seed, pname):
    """On random 8-vertex graphs the listing equals the image sets of every
    injective tuple, and its size equals the (separately pinned) count."""
    if pname not in P:
        pytest.skip(f"no pattern {pname}")
    k, e = P[pname]
    g = I.gnm_small(8, 0.6, seed)
    got = O.list_subgraphs(g, k, e)
    assert got == _edge_sets_by_permutations(g, k, e)
    assert len(got) == O.count(g, k, e)
    for s in got:
        assert len(s) == len(e)


def test_listing_size_equals_count_on_sparse_graph():
    g = I.er(200, 0.05, seed=3)
    for pname in ["house", "4-clique", "6-cycle"]:
        if pname not in P:
            continue
        k, e = P[pname]
        assert len(O.list_subgraphs(g, k, e)) == O.count(g, k, e), pname
