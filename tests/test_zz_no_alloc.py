"""gp_count_noalloc, the entry point that allocates no device memory (its
task cursor, candidate buffers and memo live in the library's static
per-GPU workspace), against gp_count through the C ABI: bit-exact on two
calls in a row, the second with a smaller input, and refusing a plan whose
buffers cannot fit the workspace."""
import pytest

from paper_2009_10955_amd import gp
from paper_2009_10955_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _noalloc(graph, plan, **launch):
    import torch
    out = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    gp.count_noalloc(graph, plan, out, **launch)
    torch.cuda.synchronize()
    c, f = out.cpu().tolist()
    assert f == 0, f
    return c & (2 ** 64 - 1)


@pytest.mark.parametrize("pname", ["house", "4-clique", "5-cycle", "triangle"])
def test_noalloc_equals_count_on_two_calls(pname):
    big = gp.Graph.from_csr(I.config_graph(2), device=True)
    small = gp.Graph.from_csr(I.er(200, 0.05, seed=3), device=True)
    k, e = I.PATTERNS[pname]
    for graph in (big, small):  # the second call has the smaller input
        plan = gp.Plan(k, e, stats=graph.stats())
        assert _noalloc(graph, plan) == gp.count(graph, plan), pname
    big.close()
    small.close()


def test_noalloc_memo_iep_and_shapes():
    """Leaf mode 4 with its memo (carved from the workspace when it fits),
    an IEP plan and narrow groups, each against gp_count, larger input first."""
    g1 = gp.Graph.from_csr(I.config_graph(2), device=True)
    g2 = gp.Graph.from_csr(I.config_graph(0), device=True)
    k, e = I.PATTERNS["5-cycle"]
    memo_plan = gp.Plan(k, e, force_order=[0, 1, 2, 3, 4],
                        force_restr=[(1, 0), (1, 2), (1, 3), (1, 4), (2, 0)])
    for graph in (g1, g2):
        for launch in (dict(group=64, leaf_mode=4, chunk=2), dict(group=16, leaf_mode=1),
                       dict(group=32, leaf_mode=3, split_ways=4, split_vertices=64)):
            assert _noalloc(graph, memo_plan, **launch) == gp.count(graph, memo_plan, **launch), launch
        for pname in ["house", "4-star"]:
            ip = gp.Plan(*I.PATTERNS[pname], stats=graph.stats(), iep=True)
            assert ip.info().iep >= 2
            assert _noalloc(graph, ip) == gp.count(graph, ip), pname
    g1.close()
    g2.close()


def test_noalloc_rejects_buffers_beyond_the_workspace():
    """K_{2,n}: two vertices of degree n, so every candidate buffer slot has
    room for n ids; with 8-lane groups one block's slots need more than the
    32 MiB workspace, and the call is refused without running."""
    import torch
    n = 400_000
    g = I.complete_bipartite(2, n)
    graph = gp.Graph.from_csr(g, device=True)
    # the 4-clique builds N(v0) & N(v1) into a buffer slot
    plan = gp.Plan(*I.PATTERNS["4-clique"], stats=graph.stats())
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(gp.GpError) as ei:
        gp.count_noalloc(graph, plan, out, group=8)
    assert ei.value.status == -7
    # the same plan with one 64-lane group per wavefront fits and counts
    assert _noalloc(graph, plan, group=64) == gp.count(graph, plan, group=64)
    graph.close()
