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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def moves_of(rs, n, k, part, count, noop=0):
    us = rs.choice(n, size=min(count, n), replace=False).astype(np.uint32)
    ts = np.array([(int(part[u]) + 1 + rs.randint(k - 1)) % k for u in us], np.uint32)
    ts[:noop] = part[us[:noop]]  # moves to the node's own block
    return us, ts


TABLE_CASES = [("multigraph", 2), ("multigraph", 64), ("hubs", 8), ("hubs", 130), ("grid2d", 200), ("rmat16", 256)]


@pytest.mark.parametrize("name,k", TABLE_CASES)
def test_graph_gain_table_and_moves_match_oracle(hgp, orc, name, k):
    H = hgp
    h = graph(name)
    G = H.Hypergraph.from_host(h)
    rs = np.random.RandomState(k)
    for kind in ("greedy", "random"):
        part = orc.greedy_ip(h, k) if kind == "greedy" else rs.randint(0, k, size=h.n).astype(np.uint32)
        print(f"[graph table] {name} k={k} {kind}", file=sys.stderr, flush=True)
        om_o = orc.graph_gain_table(h, k, part)
        t = dev(part)
        om = H.graph_gain_table(G, k, t)
        assert np.array_equal(om.cpu().numpy(), om_o)
        for count in (1, 37, h.n // 3):
            print(f"[graph moves] {name} k={k} {kind} moves={count}", file=sys.stderr, flush=True)
            us, ts = moves_of(rs, h.n, k, part, count, noop=min(3, count // 4))
            part_o, g_o, om2_o = orc.graph_moves(h, k, part, us, ts, om_o)
            t = dev(part)
            om = H.graph_gain_table(G, k, t)
            g = H.graph_moves(G, k, t, dev(us), dev(ts), omega=om)
            assert np.array_equal(t.cpu().numpy().view(np.uint32), part_o)
            assert np.array_equal(g.cpu().numpy(), g_o)
            assert np.array_equal(om.cpu().numpy(), om2_o)
            # gains only, no table
            t = dev(part)
            g = H.graph_moves(G, k, t, dev(us), dev(ts))
            assert np.array_equal(g.cpu().numpy(), g_o)


def test_graph_entry_points_reject_invalid(hgp, orc):
    H = hgp
    h = graph("grid2d")
    k = 4
    G = H.Hypergraph.from_host(h)
    part = orc.greedy_ip(h, k)
    t = dev(part)
    om = H.graph_gain_table(G, k, t)
    before = om.cpu().numpy().copy()
    for us, ts in (([5, 9, 5], [1, 2, 3]), ([5, h.n], [1, 1]), ([5, 6], [1, k])):
        with pytest.raises(H.HGPError):
            H.graph_moves(G, k, t, dev(us), dev(ts), omega=om)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), part)
    assert np.array_equal(om.cpu().numpy(), before)
    # not a graph: a net of three pins
    hx = W.from_nets(6, [[0, 1], [1, 2, 3], [4, 5]])
    Gx = H.Hypergraph.from_host(hx)
    px = dev(np.zeros(6, np.uint32))
    with pytest.raises(H.HGPError):
        H.graph_gain_table(Gx, 2, px)
    with pytest.raises(H.HGPError):
        H.graph_moves(Gx, 2, px, dev([1]), dev([1]))
