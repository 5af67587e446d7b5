"""GPU parity on graphs (every net has two pins): LP runs on the adjacency
array and the cut bits instead of net records (Sec. 10), and must still give
the oracle's partitions, objectives and block weights at every level."""
import sys

import numpy as np
import pytest

from paper_2303_17679_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_17679_amd as H
    H.lib()
    return H


def graph(name):
    rs = np.random.RandomState(31)
    if name == "multigraph":  # random edges with duplicates and weights
        n, m = 30000, 90000
        a = rs.randint(0, n, size=m)
        b = (a + 1 + rs.randint(0, n - 1, size=m)) % n
        edges = [sorted((int(x), int(y))) for x, y in zip(a, b)]
        return W.from_nets(n, edges, nwgt=rs.randint(1, 5, size=m), vwgt=rs.randint(1, 4, size=n))
    if name == "hubs":  # a few vertices adjacent to most others
        n = 20000
        edges = [[0, v] for v in range(1, n)] + [[1, v] for v in range(2, n, 3)]
        edges += [sorted(rs.choice(n, 2, replace=False).tolist()) for _ in range(30000)]
        return W.from_nets(n, edges)
    if name == "grid2d":  # a 2D mesh
        s = 150
        edges = [[y * s + x, y * s + x + 1] for y in range(s) for x in range(s - 1)]
        edges += [[y * s + x, (y + 1) * s + x] for y in range(s - 1) for x in range(s)]
        return W.from_nets(s * s, edges)
    return W.workload(name)[0]


CASES = [("multigraph", 2, 1), ("multigraph", 100, 2), ("hubs", 8, 3), ("grid2d", 16, 4), ("rmat16", 256, 5)]


@pytest.mark.parametrize("name,k,seed", CASES)
def test_graph_levels_bit_exact(hgp, orc, name, k, seed):
    import torch
    H = hgp
    h = graph(name)
    assert orc.graph_adjacency(h) is not None  # a graph
    P_or = orc.params(k, seed=seed)
    P = H.params(k, seed=seed)
    lv = orc.hierarchy(h, P_or)
    print(f"[graph {name}] levels {[L['h'].n for L in lv]}", file=sys.stderr, flush=True)
    for l, L in enumerate(lv):
        G = H.Hypergraph.from_host(L["h"])
        part_in = L["ip"] if "ip" in L else L["proj"]
        t = torch.from_numpy(np.ascontiguousarray(part_in, np.uint32).view(np.int32)).cuda()
        f, bw = H.refine_lp(G, P, l, t)
        assert f == L["f"], (l, f, L["f"])
        assert np.array_equal(t.cpu().numpy().view(np.uint32), L["part"]), l
        assert bw.cpu().numpy().tolist() == L["bw"].tolist()
    part_o, f_o, L_o = orc.partition(h, P_or)
    part, f, levels = H.partition(H.Hypergraph.from_host(h), P)
    assert (levels, f) == (L_o, f_o)
    assert np.array_equal(part.cpu().numpy().view(np.uint32), part_o)
