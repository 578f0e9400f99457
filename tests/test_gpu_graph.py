"""The fast product captured in a HIP graph (through torch.cuda.graph): every
replay must equal the eager product on the same input, with eager work and
synchronisations between replays, for one set and for a forest of uneven sets."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def imq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_04194_amd as m
    return m


def _replays_match_eager(tree, n, prec, seed):
    g = np.random.default_rng(seed)
    dt = torch.float32 if prec == "fp32" else torch.float64
    u_static = torch.tensor(g.uniform(-1, 1, n), device="cuda:0", dtype=dt)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                 # warm-up: workspaces and side streams exist
        for _ in range(2):
            tree.matvec(u_static, prec)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b_static = tree.matvec(u_static, prec)
    for rep in range(4):
        u_new = torch.tensor(g.uniform(-1, 1, n), device="cuda:0", dtype=dt)
        u_static.copy_(u_new)
        graph.replay()
        torch.cuda.synchronize()
        eager = tree.matvec(u_new, prec)
        torch.cuda.synchronize()
        assert torch.equal(b_static, eager), f"replay {rep}"
        _ = (u_new * 2).sum().item()              # unrelated eager work between replays


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_graph_replays_equal_eager_products(imq, prec):
    d = W.small(5000)
    tree = imq.build_tree(torch.tensor(d["xy"], device="cuda:0"), d["c"], leaf=32, p=10)
    _replays_match_eager(tree, 5000, prec, 3)


def test_graph_of_a_forest_of_uneven_sets(imq):
    g0 = W.rng(71, 1)
    sizes = [1500, 40, 3000, 700, 1]
    sets = [W.uniform_points(k, g0) for k in sizes]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    tree = imq.build_tree(torch.tensor(np.concatenate(sets), device="cuda:0"), [0.05, 0.1, 0.02, 0.2, 0.07],
                          leaf=32, p=10, set_offsets=list(offs))
    _replays_match_eager(tree, int(offs[-1]), "fp32", 4)
