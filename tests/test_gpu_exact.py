"""Exactness of the device accumulation, IEP in batches and serving, and the
byte-accounting instantiation: the HIP path through the C ABI against exact
integer arithmetic (Python big ints) and the CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2009_10955_amd import gp
from paper_2009_10955_amd import inputs as I

pytestmark = pytest.mark.gpu
P = I.PATTERNS
M64 = (1 << 64) - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


# ------------------------------------------------- 128-bit totals (Section II-A)

def _want(values, div):
    s = sum(int(v) for v in values)
    q, r = divmod(s, div)
    flags = (1 if q >> 64 else 0) | (2 if r else 0)
    return q & M64, flags


@pytest.mark.parametrize("case", ["max_lanes", "iep_range", "near_2_63", "random", "empty", "one"])
def test_device_sum_is_exact_in_128_bits(case):
    """The counting kernels' accumulation (lane carries, 128-bit wavefront
    sums, 128-bit device total, final division) on values no graph here
    reaches: a sum in [2^64, 2^64 * div) divided by div fits and is exact
    (an IEP total whose count fits is not an overflow); a quotient >= 2^64
    is flagged; a remainder is flagged."""
    rng = np.random.default_rng(11)
    if case == "max_lanes":
        vals = np.full(5000, M64, dtype=np.uint64)
        divs = [1, 5000, 4999, 2, 7]
    elif case == "iep_range":
        # total = 3 * (2^64 - 5): the count 2^64 - 5 fits, the total does not
        vals = np.array([M64 - 4] * 3, dtype=np.uint64)
        divs = [3, 1, 6]
    elif case == "near_2_63":
        vals = (np.uint64(1 << 63) + rng.integers(0, 1 << 20, 4097).astype(np.uint64)).astype(np.uint64)
        divs = [1, 4097, 2]
    elif case == "random":
        vals = rng.integers(0, 1 << 63, 20000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, 20000).astype(np.uint64)
        s = sum(int(v) for v in vals)
        divs = [1, 2, 3, 10, 12, 720]
        # make one divisor exact by construction
        vals = np.append(vals, np.uint64((720 - s % 720) % 720))
    elif case == "empty":
        vals = np.zeros(0, dtype=np.uint64)
        divs = [1, 6]
    else:
        vals = np.array([123456789], dtype=np.uint64)
        divs = [1, 3]
    for div in divs:
        got = gp.check_sum(vals, div)
        assert got == _want(vals, div), (case, div)


# --------------------------------------------------------- IEP in batches

def test_batch_with_iep_plans_equals_plain_and_oracle():
    """IEP plans (2, 3 and 4 inner levels) and plain plans in one launch,
    eager and replayed from a hipGraph, each plan at its own shape or at a
    common one: the oracle's counts."""
    g = I.er(60, 0.22, seed=8)
    graph = gp.Graph.from_csr(g, device=True)
    names = ["house", "4-star", "5-star", "spider", "k4-path", "4-clique", "5-cycle", "triangle",
             "6-cycle-chord"]
    plans = []
    for n in names:
        p = gp.Plan(*P[n], stats=graph.stats(), iep=True)
        plans.append(p)
    assert max(p.info().iep for p in plans) >= 3
    assert any(p.info().iep == 0 for p in plans)
    want = [O.count(g, *P[n]) for n in names]
    assert [gp.count(graph, p) for p in plans] == want
    assert gp.count_batch(graph, plans) == want
    for grp, leaf in [(64, 1), (32, 3), (16, 4)]:
        assert gp.count_batch(graph, plans, group=grp, leaf_mode=leaf) == want, (grp, leaf)
    b = gp.Batch(graph, plans)
    for _ in range(3):
        assert b.run() == want
    b.close()


def test_batch_per_plan_shapes_equal_plain():
    """Plans tuned to different launch shapes (group width, leaf mode, grab,
    split) run in one launch at their own shapes: each count equals its own
    plain launch's."""
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    names = ["house", "5-cycle", "prism", "6-clique", "k4-path"]
    tuned = [gp.Plan(*P[n], stats=graph.stats()).tuned(graph, budget_seconds=0.5) for n in names]
    shapes = {(t.launch()["group"], t.launch()["leaf_mode"]) for t in tuned}
    want = [gp.count(graph, t) for t in tuned]
    assert gp.count_batch(graph, tuned) == want, shapes
    b = gp.Batch(graph, tuned)
    assert b.run() == want
    b.close()


def test_served_iep_queries_equal_solo_counts():
    """Stars and trees served with IEP plans (the server's default) equal
    their solo counts and the oracle's."""
    g = I.er(80, 0.15, seed=4)
    graph = gp.Graph.from_csr(g, device=True)
    srv = gp.Server([graph])
    names = ["4-star", "5-star", "spider", "5-path", "house", "4-clique"]
    tickets = [srv.submit(0, *P[n]) for n in names for _ in range(3)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for i, n in enumerate([n for n in names for _ in range(3)]):
        st, c, _ = res[i]
        assert st == 0, (n, st)
        assert c == O.count(g, *P[n]), n


# ---------------------------------------------------------- byte accounting

@pytest.mark.parametrize("leaf", [1, 4])
def test_accounting_runs_the_timed_path(leaf):
    """The instrumented kernel takes the same leaf mode (and memo) as the
    timed one: its count is the count, and it reports bytes."""
    g = I.config_graph(2)
    graph = gp.Graph.from_csr(g, device=True)
    k, e = P["5-cycle"]
    plan = gp.Plan(k, e, force_order=[0, 1, 2, 3, 4], force_restr=[(1, 0), (1, 2), (1, 3), (1, 4), (2, 0)])
    want = gp.count(graph, plan, group=64, leaf_mode=leaf)
    c, b = gp.count_traffic(graph, plan, group=64, leaf_mode=leaf)
    assert c == want and b > 0
    ip = gp.Plan(*P["4-star"], stats=graph.stats(), iep=True)
    c2, b2 = gp.count_traffic(graph, ip)
    assert c2 == gp.count(graph, ip) and b2 > 0
