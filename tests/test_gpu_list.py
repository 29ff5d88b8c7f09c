"""GPU embedding listing (gp_list, through the C ABI) against the oracle's
listing of Section II-A: the same set of subgraphs, each exactly once, every
row a valid map in original vertex ids. Where the oracle's Python listing
would be slow the rows are checked by properties that fix the set at any
size: every row a valid embedding, no subgraph twice, and as many rows as the
oracle's count."""
import numpy as np
import pytest

import oracle as O
from paper_2009_10955_amd import gp
from paper_2009_10955_amd import inputs as I

pytestmark = pytest.mark.gpu
P = I.PATTERNS


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _edge_keys(g, rows: np.ndarray, edges) -> np.ndarray:
    """Per row, the sorted keys min*n + max of its image edges."""
    n = g.row_ptr.shape[0] - 1
    a = rows[:, [x for x, _ in edges]].astype(np.int64)
    b = rows[:, [y for _, y in edges]].astype(np.int64)
    return np.sort(np.minimum(a, b) * n + np.maximum(a, b), axis=1)


def _check_valid_distinct(g, rows: np.ndarray, k: int, edges) -> None:
    """Every row injective with each pattern edge on a data edge, and no two
    rows the same subgraph."""
    n = g.row_ptr.shape[0] - 1
    assert rows.ndim == 2 and rows.shape[1] == k
    if rows.shape[0] == 0:
        return
    assert rows.min() >= 0 and rows.max() < n
    srt = np.sort(rows, axis=1)
    assert (np.diff(srt, axis=1) > 0).all(), "a row repeats a vertex"
    deg = np.diff(g.row_ptr)
    adj = np.repeat(np.arange(n, dtype=np.int64), deg) * n + np.asarray(g.col, dtype=np.int64)
    for a, b in edges:
        keys = rows[:, a].astype(np.int64) * n + rows[:, b]
        assert np.isin(keys, adj).all(), f"pattern edge ({a},{b}) not on a data edge"
    ek = _edge_keys(g, rows, edges)
    assert np.unique(ek, axis=0).shape[0] == rows.shape[0], "a subgraph listed twice"


def _as_sets(g, rows: np.ndarray, edges) -> set:
    return {frozenset((min(int(r[a]), int(r[b])), max(int(r[a]), int(r[b]))) for a, b in edges) for r in rows}


def _list(graph, plan, **kw):
    rows, total = gp.list_embeddings(graph, plan, **kw)
    return rows.cpu().numpy(), total


SMALL = [("er200", lambda: I.er(200, 0.05, seed=3),
          ["edge", "triangle", "3-star", "4-path", "4-cycle", "diamond", "tailed-triangle", "house",
           "5-cycle", "k4-path", "prism", "5-wheel"]),
         ("config0", lambda: I.config_graph(0), ["triangle", "4-cycle", "house", "5-cycle"]),
         ("chunglu400", lambda: I.chung_lu(400, 2000, 2.1), ["triangle", "diamond", "4-clique", "4-cycle"])]


@pytest.mark.parametrize("gname,make,pats", SMALL, ids=[s[0] for s in SMALL])
def test_list_equals_oracle_listing(gname, make, pats):
    """The listed subgraphs are exactly the oracle's, each once, on graphs
    with and without hub bitmaps, with the planner's configuration."""
    g = make()
    graph = gp.Graph.from_csr(g, device=True)
    for pname in pats:
        k, e = P[pname]
        plan = gp.Plan(k, e, stats=graph.stats())
        rows, total = _list(graph, plan)
        want = O.list_subgraphs(g, k, e)
        assert total == len(want), pname
        _check_valid_distinct(g, rows, k, e)
        assert _as_sets(g, rows, e) == want, pname


@pytest.mark.parametrize("pname", ["house", "5-cycle", "diamond", "6-cycle-chord", "4-clique"])
def test_list_every_set_and_schedule(pname):
    """Every emitted restriction set with two schedules (different candidate
    sources, prefix buffers and cuts in the plan), with every vertex carrying a
    bitmap and with none: the oracle's listing each time."""
    g = I.er(60, 0.2, seed=8)
    want = O.list_subgraphs(g, *P[pname])
    k, e = P[pname]
    base = gp.Plan(k, e)
    scheds = base.schedules()
    rng = np.random.default_rng(2)
    for hub in ("dense", "none"):
        graph = gp.Graph.from_csr(g, hub_bitmaps=hub)
        for si in range(min(base.info().n_sets, 6)):
            for o in [scheds[int(x)] for x in rng.choice(len(scheds), min(2, len(scheds)), replace=False)]:
                plan = gp.Plan(k, e, force_order=o, force_set=si)
                rows, total = _list(graph, plan)
                assert total == len(want), (hub, si, o)
                _check_valid_distinct(g, rows, k, e)
                assert _as_sets(g, rows, e) == want, (hub, si, o)


@pytest.mark.parametrize("pname", ["house", "5-cycle", "prism", "tailed-triangle"])
def test_list_properties_on_hub_graph(pname):
    """A power-law graph with hub bitmaps and millions of embeddings: every
    row valid, no subgraph twice, and as many as the oracle counts."""
    g = I.chung_lu(400, 2000, 2.1)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P[pname]
    plan = gp.Plan(k, e, stats=graph.stats())
    want = O.count(g, k, e)
    rows, total = _list(graph, plan)
    assert total == want and rows.shape[0] == want
    _check_valid_distinct(g, rows, k, e)


def test_list_capacity_and_paging():
    """A short buffer gets the first rows of the full listing and the full
    total; the order does not depend on the grid or the queue grab; strided
    root pages are disjoint and together give the whole listing."""
    g = I.chung_lu(400, 2000, 2.1)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P["diamond"]
    plan = gp.Plan(k, e, stats=graph.stats())
    full, total = _list(graph, plan)
    want = O.count(g, k, e)
    assert total == want
    for cap in (0, 1, 63, 64, 65, total // 3, total - 1, total, total + 100):
        rows, t2 = _list(graph, plan, capacity=cap)
        assert t2 == total and rows.shape[0] == min(cap, total), cap
        assert (rows == full[:rows.shape[0]]).all(), cap
    ref = {tuple(r) for r in _edge_keys(g, full, e)}
    pages = []
    for off in range(5):
        rows, t = _list(graph, plan, root_stride=5, root_offset=off)
        assert rows.shape[0] == t
        pages.append({tuple(r) for r in _edge_keys(g, rows, e)})
    assert sum(len(p) for p in pages) == total
    assert set().union(*pages) == ref
    # other queue grabs and grid sizes list the same rows in the same order
    for kw in (dict(chunk=1, waves_per_cu=4), dict(chunk=64, waves_per_cu=1), dict(chunk=3)):
        rows, t = _list(graph, plan, **kw)
        assert t == total and rows.shape == full.shape and (rows == full).all(), kw


def test_list_edge_cases():
    """No edges, a pattern bigger than every component, k = 2 and 3 on
    ragged root counts, k = 7 and 8 paths, and IEP plans refused."""
    empty = I.csr_from_edges(6, np.zeros(0, np.int64), np.zeros(0, np.int64))
    ge = gp.Graph.from_csr(empty, device=True)
    for pname in ("edge", "triangle", "house"):
        rows, t = _list(ge, gp.Plan(*P[pname]))
        assert t == 0 and rows.shape[0] == 0
    tri = I.disjoint_union(I.complete(3), I.complete(3))
    gt = gp.Graph.from_csr(tri, device=True)
    rows, t = _list(gt, gp.Plan(*P["4-path"]))
    assert t == 0
    rows, t = _list(gt, gp.Plan(*P["triangle"]))
    assert t == 2 and _as_sets(tri, rows, P["triangle"][1]) == O.list_subgraphs(tri, *P["triangle"])
    for n in (1, 63, 64, 65, 129):
        g = I.cycle_graph(n + 2)
        graph = gp.Graph.from_csr(g, device=True)
        for pname in ("edge", "4-path"):
            k, e = P[pname]
            rows, t = _list(graph, gp.Plan(k, e))
            assert _as_sets(g, rows, e) == O.list_subgraphs(g, k, e), (n, pname)
    g = I.er(40, 0.1, seed=4)
    graph = gp.Graph.from_csr(g, device=True)
    for k in (7, 8):
        e = [(i, i + 1) for i in range(k - 1)]
        rows, t = _list(graph, gp.Plan(k, e))
        want = O.list_subgraphs(g, k, e)
        assert t == len(want)
        _check_valid_distinct(g, rows, k, e)
        assert _as_sets(g, rows, e) == want, k
    k, e = P["4-cycle"]
    iep_plan = gp.Plan(k, e, iep=True)
    if iep_plan.info().iep:
        with pytest.raises(gp.GpError):
            gp.list_embeddings(graph, iep_plan, capacity=10)


def test_list_full_size_rmat17_5clique():
    """Every 5-clique of R-MAT scale 17 (about 1e9 rows, 20 GB) in one launch:
    as many rows as the count, 100,000 sampled rows valid, one root page free
    of repeats, and for sampled rows the number of listed rows that share
    their first two schedule images equals the oracle's count of restricted
    maps with those two vertices pinned (in the oracle's own relabelling)."""
    import torch
    g = I.config_graph(1)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P["5-clique"]
    plan = gp.Plan(k, e, stats=graph.stats())
    want = gp.count(graph, plan)
    rows, total = gp.list_embeddings(graph, plan, capacity=want)
    assert total == want and tuple(rows.shape) == (want, k)
    rng = np.random.default_rng(7)
    idx = torch.from_numpy(rng.integers(0, total, 100_000)).cuda()
    _ = _check_valid_rows(g, rows[idx].cpu().numpy(), k, e)
    rp, col, new_id = O.relabel_by_degree(g)
    lay = O._CSRView(rp, col)
    order, restr = plan.order, plan.restrictions
    for r in rng.integers(0, total, 6):
        x0, x1 = int(rows[r, order[0]]), int(rows[r, order[1]])
        listed = int(((rows[:, order[0]] == x0) & (rows[:, order[1]] == x1)).sum())
        pinned = O.count_maps(lay, k, e, restr=restr, pins=[(order[0], int(new_id[x0])),
                                                             (order[1], int(new_id[x1]))])
        assert listed == pinned, (x0, x1)
    page, t = gp.list_embeddings(graph, plan, root_stride=64, root_offset=5)
    assert page.shape[0] == t
    key = torch.sort(page, dim=1).values
    assert torch.unique(key, dim=0).shape[0] == t
    del rows, page, key
    torch.cuda.empty_cache()


def _check_valid_rows(g, rows: np.ndarray, k: int, edges) -> None:
    n = g.row_ptr.shape[0] - 1
    assert rows.min() >= 0 and rows.max() < n
    assert (np.diff(np.sort(rows, axis=1), axis=1) > 0).all()
    adj = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr)) * n + np.asarray(g.col, np.int64)
    for a, b in edges:
        assert np.isin(rows[:, a].astype(np.int64) * n + rows[:, b], adj).all()
