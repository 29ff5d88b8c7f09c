"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact, on seeded graphs that span several tiles, ragged tails and the
degenerate cases."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_2009_10955_amd import gp
from paper_2009_10955_amd import inputs as I

pytestmark = pytest.mark.gpu
P = I.PATTERNS
VARIANTS = [dict(group=g, leaf_mode=l) for g in (64, 32, 16, 8) for l in (1, 2, 3, 4)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _count(graph, k, e, **kw):
    launch = {x: kw.pop(x) for x in ("group", "leaf_mode", "chunk", "waves_per_cu", "split_ways",
                                     "split_vertices") if x in kw}
    plan = gp.Plan(k, e, stats=graph.stats(), **kw)
    return gp.count(graph, plan, **launch)


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("device_input", [False, True])
def test_layout_and_stats_match_oracle(device_input):
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=device_input)
    s = graph.stats()
    assert (s.n, s.m, s.max_degree) == (g.n, g.m, int(g.degrees().max()))
    assert s.tri_cnt == 6 * O.count(g, *P["triangle"])
    rp, col, new_id = O.relabel_by_degree(g)
    assert np.array_equal(graph.new_id(), new_id)
    lrp, lcol = graph.layout()
    assert np.array_equal(lrp, rp)
    assert np.array_equal(lcol, col)


def test_bad_csr_is_rejected():
    def load(rp, col):
        with pytest.raises(gp.GpError) as ei:
            gp.Graph(np.array(rp, np.int64), np.array(col, np.int32))
        return ei.value.status
    assert load([0, 2, 3, 4], [2, 1, 0, 0]) == -2          # unsorted list
    assert load([0, 1, 1], [1]) == -3                      # asymmetric
    assert load([0, 2, 3], [0, 1, 0]) == -4                # self-loop
    assert load([0, 2, 4], [1, 1, 0, 0]) == -5             # duplicate
    assert load([0, 1, 2], [5, 0]) == -11                  # out of range
    assert load([0, 1, 3], [1, 0]) == -11                  # row_ptr[n] != nnz


def test_empty_and_edgeless_graphs():
    k, e = P["triangle"]
    for n in (1, 5):
        graph = gp.Graph(np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
        assert graph.stats().m == 0
        assert _count(graph, k, e) == 0
        assert _count(graph, *P["edge"]) == 0


# ------------------------------------------------------------ config 0

@pytest.mark.parametrize("pname", I.CONFIG_PATTERNS[0])
def test_config0_counts(pname):
    g = I.config_graph(0)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P[pname]
    want = O.count(g, k, e)
    for v in VARIANTS:
        assert _count(graph, k, e, **v) == want, v


# ------------------------------------------------------- leaf mode 4

@pytest.mark.parametrize("pname", ["4-cycle", "diamond", "house", "5-cycle", "6-cycle-chord", "prism",
                                   "k4-path", "5-wheel", "6-cycle"])
def test_flat_bitmap_leaf_every_set(pname):
    """Leaf mode 4 (long last-level lists walked by the whole group against a
    shared hub bitmap) on a graph where every vertex has a bitmap: every
    emitted restriction set with two schedules, each group width, plain, split
    and sampled, equals the oracle."""
    g = I.er(48, 0.3, seed=21)
    graph = gp.Graph.from_csr(g, hub_bitmaps="dense")
    k, e = P[pname]
    want = O.count(g, k, e)
    base = gp.Plan(k, e)
    scheds = base.schedules()
    rng = np.random.default_rng(1)
    for si in range(min(base.info().n_sets, 8)):
        for o in [scheds[int(x)] for x in rng.choice(len(scheds), min(2, len(scheds)), replace=False)]:
            plan = gp.Plan(k, e, force_order=o, force_set=si)
            for grp in (64, 32, 16, 8):
                assert gp.count(graph, plan, group=grp, leaf_mode=4) == want, (o, si, grp)
            assert gp.count(graph, plan, group=32, leaf_mode=4, split_ways=5,
                            split_vertices=1 << 20) == want
            parts = [gp.count(graph, plan, group=16, leaf_mode=4, root_stride=3, root_offset=r)
                     for r in range(3)]
            assert sum(parts) == want


@pytest.mark.parametrize("pname", ["4-cycle", "diamond", "tailed-triangle", "4-clique"])
def test_coop_leaf_long_lists(pname):
    """Leaf mode 4 where last-level lists are longer than a group walks
    alone (degree ~72, every vertex a hub), against the oracle."""
    g = I.er(120, 0.6, seed=5)
    graph = gp.Graph.from_csr(g, hub_bitmaps="dense")
    k, e = P[pname]
    want = O.count(g, k, e)
    base = gp.Plan(k, e)
    for si in range(min(base.info().n_sets, 4)):
        plan = gp.Plan(k, e, force_set=si)
        for grp in (64, 32, 16, 8):
            assert gp.count(graph, plan, group=grp, leaf_mode=4) == want, (si, grp)


def test_flat_bitmap_leaf_per_root_on_hub_graph():
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["house", "5-cycle", "4-cycle"]:
        plan = gp.Plan(*P[pname], stats=graph.stats())
        want = gp.count(graph, plan, leaf_mode=1)
        assert gp.count(graph, plan, leaf_mode=4, group=32) == want, pname
        assert gp.count(graph, plan, leaf_mode=4, group=64) == want, pname
        total, per = gp.count_per_root(graph, plan, leaf_mode=4, group=16)
        assert total == want and int(per.sum().item()) == want


# ------------------------------------------------------- split root tasks

SPLITS = [dict(split_ways=w, split_vertices=v) for w, v in
          [(1, 0), (2, 1 << 20), (3, 8), (7, 1 << 20), (64, 1 << 20), (16, 1)]]


@pytest.mark.parametrize("pname", ["4-cycle", "4-clique", "diamond", "house", "5-cycle",
                                   "6-cycle-chord", "prism", "5-wheel"])
def test_split_roots_equal_oracle(pname):
    """Heavy roots run as several tasks over disjoint slices of their
    level-2 candidates: every split, group width and leaf mode gives the
    oracle's count, also with one root per queue grab."""
    g = I.config_graph(0)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P[pname]
    want = O.count(g, k, e)
    for sp in SPLITS:
        for v in (dict(group=64, leaf_mode=1), dict(group=16, leaf_mode=2),
                  dict(group=32, leaf_mode=3, chunk=1), dict(group=8, leaf_mode=1, chunk=3),
                  dict(group=64, leaf_mode=4, chunk=1)):
            assert _count(graph, k, e, **sp, **v) == want, (sp, v)


def test_leaf4_memo_on_an_eligible_plan():
    """The 5-cycle configuration whose last level keeps per-root counts of
    hub candidates (leaf mode 4 memo): with every vertex a hub and with hubs
    by degree, every queue grab (split tasks of one root sharing a group's
    memo or not), split, group width and per-root count equals the oracle."""
    g = I.er(120, 0.3, seed=5)
    k, e = P["5-cycle"]
    want = O.count(g, k, e)
    plan = gp.Plan(k, e, force_order=[0, 1, 2, 3, 4], force_restr=[(1, 0), (1, 2), (1, 3), (1, 4), (2, 0)])
    for hub in ("dense", "auto"):
        graph = gp.Graph.from_csr(g, device=True, hub_bitmaps=hub)
        for ch in (1, 4, 16):
            for sw, sv in ((1, 0), (16, 1 << 20), (3, 8)):
                for grp in (64, 32, 16):
                    got = gp.count(graph, plan, group=grp, leaf_mode=4, chunk=ch, split_ways=sw, split_vertices=sv)
                    assert got == want, (hub, ch, sw, sv, grp)
        tot4, per4 = gp.count_per_root(graph, plan, group=64, leaf_mode=4)
        tot1, per1 = gp.count_per_root(graph, plan, group=64, leaf_mode=1)
        assert tot4 == tot1 == want and bool((per4 == per1).all()), hub


def test_split_roots_with_hubs_and_sampling():
    """A hub-heavy graph (hub bitmaps on): split counts equal unsplit ones,
    and strided root samples of a split launch still partition the count."""
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["4-cycle", "house", "5-cycle"]:
        plan = gp.Plan(*P[pname], stats=graph.stats())
        want = gp.count(graph, plan, split_ways=1)
        for ways, verts in [(16, 256), (5, 1 << 20), (128, 4)]:
            assert gp.count(graph, plan, split_ways=ways, split_vertices=verts) == want, (pname, ways)
            for ch in (1, 2):
                assert gp.count(graph, plan, group=64, leaf_mode=4, chunk=ch, split_ways=ways,
                                split_vertices=verts) == want, (pname, ways, ch)
        parts = [gp.count(graph, plan, root_stride=5, root_offset=o, split_ways=9,
                          split_vertices=1 << 20) for o in range(5)]
        assert sum(parts) == want, pname


def test_split_roots_iep():
    g = I.config_graph(0)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["house", "k4-path", "6-cycle-chord"]:
        k, e = P[pname]
        plan = gp.Plan(k, e, stats=graph.stats(), iep=True)
        assert plan.info().iep >= 2
        want = O.count(g, k, e)
        for sp in SPLITS:
            assert gp.count(graph, plan, group=64, **sp) == want, (pname, sp)


def test_bad_split_is_rejected():
    graph = gp.Graph.from_csr(I.config_graph(0), device=True)
    plan = gp.Plan(*P["house"], stats=graph.stats())
    for bad in (dict(split_ways=-1), dict(split_ways=5000), dict(split_vertices=-3)):
        with pytest.raises(gp.GpError) as ei:
            gp.count(graph, plan, **bad)
        assert ei.value.status == -1


# ------------------------------------------------------------- closed forms

def test_closed_forms():
    kn = gp.Graph.from_csr(I.complete(12))
    for pname in ["triangle", "4-cycle", "4-clique", "house", "5-clique", "6-clique", "prism",
                  "5-wheel", "6-cycle"]:
        k, e = P[pname]
        aut = len(O.automorphisms(k, e))
        assert _count(kn, k, e) == math.comb(12, k) * math.factorial(k) // aut, pname
    kab = gp.Graph.from_csr(I.complete_bipartite(9, 13))
    assert _count(kab, *P["4-cycle"]) == math.comb(9, 2) * math.comb(13, 2)
    assert _count(kab, *P["triangle"]) == 0
    q = gp.Graph.from_csr(I.hypercube(8))
    assert _count(q, *P["4-cycle"]) == math.comb(8, 2) * 2 ** 6
    c = gp.Graph.from_csr(I.cycle_graph(5))
    assert _count(c, *P["5-cycle"]) == 1


@pytest.mark.parametrize("hubs", ["auto", "none", "dense"])
def test_hub_star_ragged(hubs):
    """A hub of degree 2000 (many tiles plus a ragged tail) with its leaves
    partly connected: exercises long lists and large candidate buffers."""
    rng = np.random.default_rng(3)
    s = 2000
    src = [0] * s + list(rng.integers(1, s + 1, 1500))
    dst = list(range(1, s + 1)) + list(rng.integers(1, s + 1, 1500))
    g = I.csr_from_edges(s + 1, np.array(src), np.array(dst))
    graph = gp.Graph.from_csr(g, hub_bitmaps=hubs)
    st = graph.stats()
    if hubs == "none":
        assert st.hub_vertices == 0
    elif hubs == "dense":
        assert st.hub_vertices == int((g.degrees() > 0).sum())
    else:
        assert st.hub_vertices == int((g.degrees() >= 64).sum())
    for pname in ["triangle", "4-cycle", "tailed-triangle", "diamond", "4-clique"]:
        k, e = P[pname]
        want = O.count(g, k, e)
        for v in VARIANTS[::3] + [dict(group=64, leaf_mode=4), dict(group=8, leaf_mode=4)]:
            assert _count(graph, k, e, **v) == want, (pname, v)
    # stars: closed form sum over vertices of C(deg, 3)
    star = sum(math.comb(int(d), 3) for d in g.degrees())
    for v in VARIANTS:
        assert _count(graph, *P["3-star"], **v) == star, v


# ------------------------------------------------------- every pattern, graphs

@pytest.mark.parametrize("seed,hubs", [(101, "none"), (102, "dense")])
@pytest.mark.parametrize("pname", list(P))
def test_all_patterns_random_graphs(seed, hubs, pname):
    g = I.er(60, 0.25, seed=seed)
    graph = gp.Graph.from_csr(g, hub_bitmaps=hubs)
    k, e = P[pname]
    want = O.count(g, k, e)
    for v in VARIANTS:
        assert _count(graph, k, e, **v) == want, v


@pytest.mark.parametrize("pname", ["triangle", "4-cycle", "4-clique", "diamond", "house",
                                   "5-cycle", "6-cycle-chord", "k4-path", "tailed-triangle"])
def test_every_restriction_set_and_schedule(pname):
    """Each emitted set with several efficient schedules gives the oracle count."""
    g = I.er(40, 0.3, seed=7)
    graph = gp.Graph.from_csr(g)
    k, e = P[pname]
    want = O.count(g, k, e)
    base = gp.Plan(k, e)
    scheds = base.schedules()
    n_sets = base.info().n_sets
    rng = np.random.default_rng(0)
    for si in range(n_sets):
        for o in [scheds[int(x)] for x in rng.choice(len(scheds), min(3, len(scheds)), replace=False)]:
            plan = gp.Plan(k, e, force_order=o, force_set=si)
            assert gp.count(graph, plan, group=16) == want, (o, si)


def test_random_patterns_up_to_six_vertices():
    rng = np.random.default_rng(5)
    g = I.er(45, 0.3, seed=9)
    graph = gp.Graph.from_csr(g)
    for _ in range(25):
        k = int(rng.integers(3, 7))
        e = I.random_connected_pattern(k, rng, 0.5)
        assert _count(graph, k, e) == O.count(g, k, e), (k, e)


def test_relabel_and_union_invariance():
    g = I.er(80, 0.15, seed=4)
    h = I.er(70, 0.2, seed=5)
    u = I.disjoint_union(g, h)
    pu = I.permute(u, np.random.default_rng(1).permutation(u.n))
    gg, gh, gu = (gp.Graph.from_csr(x) for x in (g, h, pu))
    for pname in ["triangle", "4-cycle", "house", "5-cycle"]:
        k, e = P[pname]
        assert _count(gu, k, e) == _count(gg, k, e) + _count(gh, k, e)


# ------------------------------------------------------------ per-root parity

def _per_root_check(g, graph, pname, n_samples, seed, max_check=2_000_000, **launch):
    k, e = P[pname]
    plan = gp.Plan(k, e, stats=graph.stats())
    total, per = gp.count_per_root(graph, plan, **launch)
    per = per.cpu().numpy()
    assert int(per.sum()) == total
    assert gp.count(graph, plan, **launch) == total
    rp, col, _ = O.relabel_by_degree(g)
    lay = O._CSRView(rp, col)
    order = plan.order
    restr = plan.restrictions
    rng = np.random.default_rng(seed)
    nz = np.nonzero(per)[0]
    picks = list(rng.choice(len(col), n_samples, replace=False))
    # nonzero roots light enough for the oracle to redo within seconds,
    # including the heaviest of those
    light = nz[per[nz] <= max_check]
    if light.size:
        picks += list(rng.choice(light, min(n_samples, light.size), replace=False))
        picks.append(int(light[np.argmax(per[light])]))
    src = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    for idx in picks:
        v0, v1 = int(src[idx]), int(col[idx])
        want = O.count_maps(lay, k, e, restr=restr, pins=[(order[0], v0), (order[1], v1)],
                            threads=1)
        assert int(per[idx]) == want, (pname, idx, v0, v1)
    return total


@pytest.mark.parametrize("pname", ["triangle", "4-cycle", "4-clique", "house", "5-cycle"])
def test_per_root_counts_config2(pname):
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True, hub_bitmaps="dense" if pname == "5-cycle" else "auto")
    _per_root_check(g, graph, pname, 20, 1)


@pytest.mark.parametrize("pname", I.CONFIG_PATTERNS[1])
def test_per_root_counts_config1_full_size(pname):
    """R-MAT scale 17 at full size, default launch and leaf mode 4: per-root
    counts on sampled roots (random, nonzero, and the heaviest) equal the
    oracle's pinned counts."""
    g = I.config_graph(1)
    graph = gp.Graph.from_csr(g, device=True)
    _per_root_check(g, graph, pname, 6, 2)
    _per_root_check(g, graph, pname, 3, 3, group=64, leaf_mode=4)


def test_config2_small_patterns_full_count():
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["triangle", "4-clique", "diamond"]:
        k, e = P[pname]
        assert _count(graph, k, e) == O.count(g, k, e), pname


# ------------------------------------------------------------------ batched

@pytest.mark.parametrize("group", [64, 32, 16])
def test_batch_equals_plain(group):
    g = I.er(200, 0.08, seed=11)
    graph = gp.Graph.from_csr(g)
    names = ["triangle", "4-cycle", "house", "5-cycle", "6-cycle-chord", "prism", "edge",
             "3-star", "5-wheel"]
    plans = [gp.Plan(*P[x], stats=graph.stats()) for x in names]
    plain = [gp.count(graph, p) for p in plans]
    assert gp.count_batch(graph, plans, group=group) == plain
    assert plain == [O.count(g, *P[x]) for x in names]


def test_batch_mixed_sizes_up_to_eight():
    g = I.er(24, 0.6, seed=3)
    graph = gp.Graph.from_csr(g, hub_bitmaps="dense")
    pats = [P["edge"], P["triangle"], P["diamond"], P["5-clique"], P["prism"],
            (7, [(i, j) for i, j in itertools.combinations(range(7), 2)]),
            (8, [(i, (i + 1) % 8) for i in range(8)] + [(0, 4)]),
            (7, [(i, i + 1) for i in range(6)] + [(0, 6), (2, 5)])]
    plans = [gp.Plan(k, e, stats=graph.stats()) for k, e in pats]
    want = [O.count(g, k, e) for k, e in pats]
    assert [gp.count(graph, p) for p in plans] == want
    assert gp.count_batch(graph, plans) == want


def test_batch_graph_replays_match_eager():
    """The captured hipGraph replays several times, with eager counts and
    synchronisations in between; every replay equals the eager result."""
    import torch
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    names = ["triangle", "4-cycle", "diamond", "house", "4-clique", "tailed-triangle"]
    plans = [gp.Plan(*P[x], stats=graph.stats()) for x in names]
    eager = [gp.count(graph, p) for p in plans]
    batch = gp.Batch(graph, plans)
    for rep in range(4):
        assert batch.run() == eager, rep
        assert gp.count(graph, plans[rep % len(plans)]) == eager[rep % len(plans)]
        torch.cuda.synchronize()
    batch.close()


def test_batch_of_sixty_four_plans():
    g = I.er(120, 0.12, seed=21)
    graph = gp.Graph.from_csr(g)
    rng = np.random.default_rng(8)
    pats = []
    for _ in range(64):
        k = int(rng.integers(2, 6))
        pats.append((k, I.random_connected_pattern(k, rng, 0.5)))
    plans = [gp.Plan(k, e, stats=graph.stats()) for k, e in pats]
    want = [gp.count(graph, p) for p in plans]
    assert gp.count_batch(graph, plans) == want
    assert want[:8] == [O.count(g, k, e) for k, e in pats[:8]]


# ------------------------------------------------------- sampling and tuning

def test_root_sampling_partitions_the_count():
    """Strided root samples over all offsets add up to the full count."""
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["4-cycle", "house", "4-clique"]:
        plan = gp.Plan(*P[pname], stats=graph.stats())
        total = gp.count(graph, plan)
        stride = 7
        parts = [gp.count(graph, plan, root_stride=stride, root_offset=o) for o in range(stride)]
        assert sum(parts) == total, pname
        assert gp.count(graph, plan, root_stride=1, root_offset=10 ** 9) == 0


def test_tuned_plans_count_the_same():
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["triangle", "4-cycle", "diamond", "4-clique", "house", "5-cycle"]:
        k, e = P[pname]
        plan = gp.Plan(k, e, stats=graph.stats())
        tuned = plan.tuned(graph, budget_seconds=2.0)
        inf = tuned.info()
        assert inf.tuned == 1 and inf.n_measured >= 1
        r = frozenset(tuned.restrictions)
        assert O.validate(k, e, r)
        want = gp.count(graph, plan)
        assert gp.count(graph, tuned) == want, pname
        if pname in ("triangle", "4-clique", "diamond"):
            assert want == O.count(g, k, e)
        # cached second call gives the same configuration
        again = plan.tuned(graph)
        assert again.order == tuned.order and again.restrictions == tuned.restrictions


def test_tuning_with_iep_candidates_counts_the_same():
    """With IEP configurations in the race the tuned plan (plain or IEP)
    still gives the oracle's count; an IEP winner is refused by listing."""
    g = I.config_graph(0)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["3-star", "4-path", "house", "k4-path", "5-cycle", "tailed-triangle"]:
        k, e = P[pname]
        plan = gp.Plan(k, e, stats=graph.stats())
        tuned = plan.tuned(graph, budget_seconds=1.0, try_iep=True)
        want = O.count(g, k, e)
        assert gp.count(graph, tuned) == want, pname
        for grp in (64, 32):
            assert gp.count(graph, tuned, group=grp) == want, (pname, grp)
        if tuned.info().iep:
            assert tuned.info().iep_div >= 1
            with pytest.raises(gp.GpError):
                gp.list_embeddings(graph, tuned, capacity=1)
        plain = plan.tuned(graph, budget_seconds=1.0)
        assert not plain.info().iep and gp.count(graph, plain) == want, pname


# ------------------------------------------------------------------ serving

@pytest.mark.parametrize("leaf", [1, 4])
def test_serving_counts_equal_solo_counts(leaf):
    """A Poisson stream of random connected 3-5-vertex patterns over two
    resident graphs, with tiny slices so queries span several iterations and
    newcomers join launches already under way: every count equals the solo
    count (and the oracle's on the small graph)."""
    from paper_2009_10955_amd import serve
    g0 = I.config_graph(0)
    g1 = I.er(300, 0.06, seed=13)
    graphs = [gp.Graph.from_csr(g0), gp.Graph.from_csr(g1, hub_bitmaps="dense")]
    pats = I.connected_patterns(3, 5)
    stream = I.poisson_stream(150, 2000.0, 2, len(pats), seed=7)
    srv = gp.Server(graphs, target_ms=2.0, initial_slice=32, leaf_mode=leaf)
    res = serve.run_stream(srv, stream, pats)
    stats = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res)
    solo = {}
    for r in res:
        key = (r["graph"], r["pattern"])
        if key not in solo:
            k, e = pats[r["pattern"]]
            solo[key] = gp.count(graphs[r["graph"]], gp.Plan(k, e, stats=graphs[r["graph"]].stats()))
        assert r["count"] == solo[key], key
    for (gi, pi), c in list(solo.items())[:12]:
        if gi == 1:
            k, e = pats[pi]
            assert c == O.count(g1, k, e)
    assert stats["completed"] == len(stream)
    assert stats["iterations"] > 1
    assert stats["joined_midflight"] > 0
    assert stats["max_batch"] > 1
    summ = serve.summarise(res)
    assert summ["completed"] == len(stream)


def test_serving_rejects_over_budget_and_reports_overflow_free():
    from paper_2009_10955_amd import serve
    graphs = [gp.Graph.from_csr(I.config_graph(0))]
    pats = [P["triangle"], P["5-clique"]]
    srv = gp.Server(graphs, cost_cap=1.0)
    t = [srv.submit(0, *p) for p in pats]
    out = [srv.wait(x) for x in t]
    srv.close()
    assert [o[0] for o in out] == [-10, -10]
    srv = gp.Server(graphs)
    out = [srv.wait(srv.submit(0, *p)) for p in pats]
    srv.close()
    assert [o[0] for o in out] == [0, 0]
    assert out[0][1] == 157


def test_serving_measured_admission():
    """max_query_ms: with a generous limit every query runs and equals its
    solo count; with a tiny limit on a hub-heavy graph the heavy pattern is
    rejected (GP_ERR_BUDGET) while the light one still completes."""
    g2 = I.config_graph(2)
    graphs = [gp.Graph.from_csr(I.config_graph(0)), gp.Graph.from_csr(g2)]
    pats = [P["triangle"], P["house"], P["5-cycle"]]
    srv = gp.Server(graphs, max_query_ms=60_000)
    t = [(gi, p, srv.submit(gi, *p)) for gi in (0, 1) for p in pats]
    out = [(gi, p, srv.wait(x)) for gi, p, x in t]
    srv.close()
    for gi, p, (st, c, _) in out:
        assert st == 0
        assert c == gp.count(graphs[gi], gp.Plan(*p, stats=graphs[gi].stats()))
    srv = gp.Server(graphs, max_query_ms=1e-3)
    st_heavy = srv.wait(srv.submit(1, *P["5-cycle"]))[0]
    srv.close()
    assert st_heavy == -10


def test_estimate_is_sane():
    """gp_estimate: positive, finite without a budget, and its sample count
    times the stride is within 3x of the full count on a power-law graph."""
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["house", "4-clique", "5-cycle"]:
        plan = gp.Plan(*P[pname], stats=graph.stats())
        e = gp.estimate(graph, plan)
        assert 0 < e["ms"] < 1e6 and e["sample_stride"] >= 1
        full = gp.count(graph, plan)
        assert full / 3 <= e["sample_count"] * e["sample_stride"] <= full * 3, pname
        e2 = gp.estimate(graph, plan, budget_ms=1e-4)
        assert e2["ms"] == float("inf") or e2["ms"] > 0
    # IEP plans are estimated too (the sample's total divided without a check)
    for pname in ["house", "4-star"]:
        iep = gp.Plan(*P[pname], stats=graph.stats(), iep=True)
        assert iep.info().iep >= 2
        e = gp.estimate(graph, iep)
        full = gp.count(graph, iep)
        assert 0 < e["ms"] < 1e6
        assert full / 3 <= e["sample_count"] * e["sample_stride"] <= full * 3, pname


def test_batch_tune_picks_a_shape_with_the_same_counts():
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    plans = [gp.Plan(*P[n], stats=graph.stats()) for n in ["house", "4-clique", "prism"]]
    want = [gp.count(graph, p) for p in plans]
    shape, ms = gp.batch_tune(graph, plans)
    # all zero: every plan at its own shape; else one shape for all
    assert (shape["group"], shape["leaf_mode"]) == (0, 0) or (
        shape["group"] in (64, 32, 16) and shape["leaf_mode"] in (1, 3, 4))
    assert ms > 0
    assert gp.count_batch(graph, plans, **shape) == want
    for grp in (16, 32, 64):
        for leaf in (1, 3, 4):
            assert gp.count_batch(graph, plans, group=grp, leaf_mode=leaf) == want, (grp, leaf)


def test_batch_with_split_roots_equals_plain():
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    plans = [gp.Plan(*P[n], stats=graph.stats()) for n in ["house", "5-cycle", "4-clique", "triangle"]]
    want = [gp.count(graph, p, split_ways=1) for p in plans]
    for ways, verts in [(1, 0), (16, 256), (7, 1 << 20)]:
        for grp, leaf in [(64, 3), (32, 1)]:
            got = gp.count_batch(graph, plans, group=grp, leaf_mode=leaf, split_ways=ways,
                                 split_vertices=verts)
            assert got == want, (ways, verts, grp, leaf)
    b = gp.Batch(graph, plans, split_ways=5, split_vertices=1 << 20)
    for _ in range(3):
        assert b.run() == want
    b.close()


@pytest.mark.parametrize("hubs", ["auto", "dense"])
def test_batch_per_plan_shapes_equal_oracle(hubs):
    """Plans of one batch at different launch shapes (every group width, leaf
    modes 1/3/4, IEP depths 2 and 3, several plans per shape and shapes
    interleaved in the caller's order): one launch per shape, counts equal to
    the oracle, eager and replayed from the captured hipGraph."""
    import torch
    g = I.er(160, 0.1, seed=12)
    graph = gp.Graph.from_csr(g, device=True, hub_bitmaps=hubs)
    st = graph.stats()
    spec = [("triangle", dict(group=8, leaf_mode=1)), ("house", dict(group=64, leaf_mode=4)),
            ("4-cycle", dict(group=16, leaf_mode=3)), ("5-cycle", dict(group=32, leaf_mode=1)),
            ("house", dict(group=32, leaf_mode=1), 2), ("prism", dict(group=8, leaf_mode=4)),
            ("4-star", dict(group=64), 3), ("6-cycle-chord", dict(group=16, leaf_mode=4)),
            ("diamond", dict(group=8, leaf_mode=1)), ("4-clique", dict(group=64, leaf_mode=4)),
            ("4-path", dict(group=64), 2), ("5-wheel", dict(group=32, leaf_mode=3))]
    plans, want = [], []
    for item in spec:
        name, launch = item[0], item[1]
        iep = item[2] if len(item) > 2 else False
        p = gp.Plan(*P[name], stats=st, iep=iep).with_launch(**launch)
        if iep:
            assert p.info().iep == iep, name
        plans.append(p)
        want.append(O.count(g, *P[name]))
    assert [gp.count(graph, p) for p in plans] == want
    assert gp.count_batch(graph, plans) == want
    b = gp.Batch(graph, plans)
    for rep in range(3):
        assert b.run() == want, rep
        assert gp.count(graph, plans[rep]) == want[rep]
        torch.cuda.synchronize()
    # strided samples of the same batch add up to the counts; an IEP plan's
    # sample quotients are rounded down, so its parts fall short by under one
    # per part
    parts = []
    for r in range(3):
        b.set_sample(3, r)
        parts.append(b.run())
    for i, (p, x) in enumerate(zip(plans, zip(*parts))):
        if p.info().iep_div > 1:
            assert want[i] - 3 < sum(x) <= want[i], (spec[i], x)
        else:
            assert sum(x) == want[i], (spec[i], x)
    b.set_sample(1, 0)
    assert b.run() == want
    b.close()


@pytest.mark.parametrize("pname", ["triangle", "4-clique", "house", "5-cycle"])
def test_xcd_task_blocks_equal_oracle(pname):
    """Tasks dealt to the XCDs in blocks (any block size, rounded up to the
    grab; ragged last round; XCDs that run dry help the others) count every
    task once: plain, sampled, split, per root and with byte accounting."""
    g = I.er(400, 0.04, seed=17)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P[pname]
    want = O.count(g, k, e)
    plan = gp.Plan(k, e, stats=graph.stats())
    for xt in (1, 7, 64, 500, 1 << 20):
        for grp, chunk in ((64, 4), (16, 3), (8, 1)):
            assert gp.count(graph, plan, group=grp, chunk=chunk, xcd_tasks=xt) == want, (xt, grp, chunk)
        assert sum(gp.count(graph, plan, xcd_tasks=xt, root_stride=5, root_offset=r) for r in range(5)) == want
        assert gp.count(graph, plan, xcd_tasks=xt, split_ways=7, split_vertices=1 << 20) == want
    total, per = gp.count_per_root(graph, plan, xcd_tasks=64)
    assert total == want and int(per.cpu().numpy().sum()) == want * (plan.info().iep_div or 1)
    c, b = gp.count_traffic(graph, plan, xcd_tasks=64)
    assert c == want and b == gp.count_traffic(graph, plan, xcd_tasks=-1)[1]


# --------------------------------------------------------------------- IEP

@pytest.mark.parametrize("pname", ["house", "diamond", "tailed-triangle", "4-path", "3-star",
                                   "prism", "6-cycle-chord", "k4-path", "5-wheel", "4-star", "5-star",
                                   "6-star", "5-path", "spider"])
@pytest.mark.parametrize("hubs", ["dense", "none"])
def test_iep_counts_equal_oracle(pname, hubs):
    """Counting the innermost 2, 3 or 4 levels with inclusion-exclusion gives
    the oracle's count, for the chosen configuration at every depth allowed
    and for every eligible configuration of a few schedules, in both IEP
    group sizes, with membership by bitmap and by binary search."""
    g = I.er(50, 0.25, seed=31)
    graph = gp.Graph.from_csr(g, hub_bitmaps=hubs)
    k, e = P[pname]
    want = O.count(g, k, e)
    depths = set()
    for cap in (2, 3, 4):
        plan = gp.Plan(k, e, stats=graph.stats(), iep=cap)
        n = plan.info().iep
        assert 2 <= n <= cap
        depths.add(n)
        for grp in (64, 32):
            assert gp.count(graph, plan, group=grp) == want, (cap, grp)
    base = gp.Plan(k, e)
    scheds = base.schedules()
    n_sets = base.info().n_sets
    checked = 0
    for o in scheds[:4]:
        for si in range(min(n_sets, 6)):
            for cap in (2, 4):
                p2 = gp.Plan(k, e, force_order=o, force_set=si, iep=cap)
                if p2.info().iep:
                    depths.add(p2.info().iep)
                    assert gp.count(graph, p2) == want, (o, si, cap)
                    checked += 1
    assert checked > 0
    if pname in ("4-star", "5-star", "6-star", "spider"):
        assert max(depths) >= 3, depths


def test_iep_per_root_and_config2():
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    for pname in ["house", "diamond"]:
        k, e = P[pname]
        plain = gp.count(graph, gp.Plan(k, e, stats=graph.stats()))
        ip = gp.Plan(k, e, stats=graph.stats(), iep=True)
        assert gp.count(graph, ip) == plain
        total, per = gp.count_per_root(graph, ip)
        assert total == plain
        assert int(per.cpu().numpy().sum()) == plain * ip.info().iep_div
    assert gp.count(graph, gp.Plan(*P["diamond"])) == O.count(g, *P["diamond"])


def test_batch_with_a_launch_per_plan_equals_oracle():
    """batch_runs = 2: every plan its own launch inside the batch (the plain
    kernel for whole plans), against the oracle and the shared-launch batch,
    eager, replayed and sampled."""
    g = I.er(160, 0.1, seed=13)
    graph = gp.Graph.from_csr(g, device=True)
    names = ["triangle", "4-cycle", "house", "5-cycle", "diamond", "prism"]
    plans = [gp.Plan(*P[n], stats=graph.stats()) for n in names]
    want = [O.count(g, *P[n]) for n in names]
    assert gp.count_batch(graph, plans, batch_runs=2) == want
    assert gp.count_batch(graph, plans, batch_runs=1) == want
    b = gp.Batch(graph, plans, batch_runs=2)
    for _ in range(2):
        assert b.run() == want
    parts = []
    for r in range(4):
        b.set_sample(4, r)
        parts.append(b.run())
    assert [sum(x) for x in zip(*parts)] == want
    b.close()


def test_iep_hub_memo_equals_oracle():
    """Inner sets of IEP plans left unbuilt as N(a) & N(x) with x a hub have
    their sizes kept in a table shared by every group of the launch: a graph
    of a few hubs with shared neighbourhoods (many bindings, in many groups,
    reach the same hub pair) counts the same as the oracle with hubs and
    without, per root, and in batches that give each plan its own launch
    (the table shared across launches). A second graph counted after the
    first, on the same device, starts from a cleared table."""
    rng = np.random.default_rng(7)
    n, hubs, deg = 300, 4, 150
    src, dst = [], []
    for h in range(hubs):
        nb = rng.choice(np.arange(hubs, n), size=deg, replace=False)
        src += [h] * deg
        dst += list(nb)
        src += [h] * (hubs - 1 - h)
        dst += list(range(h + 1, hubs))
    src += list(rng.integers(hubs, n, 600))
    dst += list(rng.integers(hubs, n, 600))
    g = I.csr_from_edges(n, np.array(src), np.array(dst))
    names = ["house", "4-path", "tailed-triangle", "k4-path", "diamond"]
    want = [O.count(g, *P[x]) for x in names]
    k, e = P["house"]
    forced = dict(force_order=(0, 1, 2, 3, 4), force_restr=[(1, 0)], iep=True)
    for hub in ("auto", "none"):
        graph = gp.Graph.from_csr(g, device=True, hub_bitmaps=hub)
        st = graph.stats()
        assert (st.hub_vertices > 0) == (hub == "auto")
        plans = [gp.Plan(*P[x], stats=st, iep=True) for x in names]
        plans.append(gp.Plan(k, e, stats=st, **forced))
        ws = want + [want[0]]
        for p, w in zip(plans, ws):
            for grp in (64, 32):
                assert gp.count(graph, p, group=grp, leaf_mode=1) == w, (hub, grp)
            tot, per = gp.count_per_root(graph, p)
            assert tot == w and int(per.cpu().numpy().sum()) == w * p.info().iep_div
        assert gp.count_batch(graph, plans, batch_runs=2) == ws
        b = gp.Batch(graph, plans, batch_runs=2)
        for _ in range(3):
            assert b.run() == ws
        b.close()
        graph.close()
    g2 = I.er(200, 0.08, seed=21)
    graph = gp.Graph.from_csr(g2, device=True, hub_bitmaps="dense")
    p2 = gp.Plan(k, e, stats=graph.stats(), **forced)
    assert gp.count(graph, p2, group=64, leaf_mode=1) == O.count(g2, k, e)
    graph.close()
