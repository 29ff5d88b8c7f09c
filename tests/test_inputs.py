"""Seeded input generators: shapes, determinism and the pattern classes."""
import itertools

import numpy as np

import oracle as O
from paper_2009_10955_amd import inputs as I


def test_generators_are_deterministic_and_canonical():
    for g, h in [(I.er(300, 0.05, 3), I.er(300, 0.05, 3)), (I.rmat(10, 8, seed=2), I.rmat(10, 8, seed=2)),
                 (I.chung_lu(500, 3000, 2.1, 3), I.chung_lu(500, 3000, 2.1, 3))]:
        assert g.sha256() == h.sha256()
        for v in range(g.n):
            nb = g.neighbors(v)
            assert np.all(np.diff(nb) > 0) and v not in nb
        src = np.repeat(np.arange(g.n), g.degrees())
        assert sorted(zip(src.tolist(), g.col.tolist())) == sorted(zip(g.col.tolist(), src.tolist()))


def test_config_graph_shapes():
    g0 = I.config_graph(0)
    assert (g0.n, g0.m) == (1000, 5017)
    g2 = I.config_graph(2)
    assert g2.n == 7000 and 95_000 < g2.m < 105_000


def test_connected_pattern_classes():
    """Connected graphs up to isomorphism: 2, 6, 21, 112 on 3..6 vertices
    (OEIS A001349); each representative connected, no two isomorphic."""
    ps = I.connected_patterns(3, 6)
    assert [sum(1 for k, _ in ps if k == j) for j in range(3, 7)] == [2, 6, 21, 112]
    for k in (3, 4, 5):
        group = [e for kk, e in ps if kk == k]
        forms = set()
        for e in group:
            es = {frozenset(x) for x in e}
            best = min(tuple(sorted(tuple(sorted((p[a], p[b]))) for a, b in e))
                       for p in itertools.permutations(range(k)))
            forms.add(best)
            # connected: a search from vertex 0 reaches every vertex
            seen, todo = {0}, [0]
            while todo:
                u = todo.pop()
                for a, b in e:
                    for x, y in ((a, b), (b, a)):
                        if x == u and y not in seen:
                            seen.add(y)
                            todo.append(y)
            assert seen == set(range(k)), e
            assert len(es) == len(e)
        assert len(forms) == len(group)


def test_poisson_stream():
    s = I.poisson_stream(2000, 50.0, 3, 141, 5)
    t = np.array([x[0] for x in s])
    assert np.all(np.diff(t) > 0)
    assert 35 < t[-1] < 45
    assert {x[1] for x in s} == {0, 1, 2}
    assert s == I.poisson_stream(2000, 50.0, 3, 141, 5)
