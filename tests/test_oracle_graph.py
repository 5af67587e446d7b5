"""Pins of the graph rules (Sec. 10) in the oracle: on hypergraphs whose nets
all have two pins, the gain w(u, V_t) - w(u, V_Pi[u]) read from one adjacency
array equals the connectivity gain and the brute-force objective change, the
edge cut equals the connectivity objective, and contraction removes
self-loops and merges parallel edges with their weights summed.  No GPU."""
import numpy as np
import pytest

import bruteforce as bf
from paper_2303_17679_amd import workloads as W


def random_graph(seed, n=14, m=30, parallel=True):
    """Random multigraph without self-loops: duplicate edges when `parallel`."""
    rs = np.random.RandomState(seed)
    edges = []
    while len(edges) < m:
        a, b = sorted(rs.choice(n, 2, replace=False).tolist())
        if parallel or (a, b) not in edges:
            edges.append((a, b))
    return W.from_nets(n, edges, nwgt=rs.randint(1, 6, size=m)), edges


@pytest.mark.parametrize("seed", range(10))
def test_adjacency_is_the_other_endpoint(orc, seed):
    h, edges = random_graph(seed)
    adj, adjw = orc.graph_adjacency(h)
    for u in range(h.n):
        got = sorted(zip(adj[h.inc_off[u]:h.inc_off[u + 1]].tolist(), adjw[h.inc_off[u]:h.inc_off[u + 1]].tolist()))
        want = sorted([(b if a == u else a, int(h.nwgt[e])) for e, (a, b) in enumerate(edges) if u in (a, b)])
        assert got == want
    # not a graph: a net of three pins
    assert orc.graph_adjacency(W.from_nets(4, [[0, 1], [1, 2, 3]])) is None


@pytest.mark.parametrize("seed", range(10))
def test_graph_gain_equals_connectivity_gain(orc, seed):
    h, edges = random_graph(seed)
    adj, adjw = orc.graph_adjacency(h)
    rs = np.random.RandomState(50 + seed)
    for k in (2, 3, 5):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        # edge cut by sets = connectivity objective (lambda - 1 is 0 or 1)
        cut = sum(int(w) for (a, b), w in zip(edges, h.nwgt) if part[a] != part[b])
        assert orc.graph_cut(h, part) == cut == orc.objective(h, k, part)[0]
        for u in range(h.n):
            for t in range(k):
                if t == part[u]:
                    continue
                g = orc.graph_gain(h, adj, adjw, part, u, t)
                assert g == orc.gain(h, part, u, t) == bf.move_delta(h, part, u, t), (u, t)


@pytest.mark.parametrize("seed", range(10))
def test_graph_contraction_drops_self_loops_and_merges_parallel_edges(orc, seed):
    h, edges = random_graph(seed, n=16, m=40)
    rs = np.random.RandomState(80 + seed)
    reps = sorted(rs.choice(16, 7, replace=False).tolist())
    rep = np.array([v if v in reps else reps[rs.randint(len(reps))] for v in range(16)], np.uint32)
    cid, H = orc.contract(h, rep)
    want = {}
    for (a, b), w in zip(edges, h.nwgt):
        ca, cb = int(cid[a]), int(cid[b])
        if ca == cb:
            continue  # self-loop
        key = (min(ca, cb), max(ca, cb))
        want[key] = want.get(key, 0) + int(w)
    got = {}
    for e in range(H.m):
        p = H.pins[H.pin_off[e]:H.pin_off[e + 1]].tolist()
        assert len(p) == 2 and p[0] < p[1]  # still a graph
        assert tuple(p) not in got  # no parallel edges left
        got[tuple(p)] = int(H.nwgt[e])
    assert got == want
    # the coarse level is a graph: its adjacency exists and its gains are the graph gains
    adj, adjw = orc.graph_adjacency(H)
    part = rs.randint(0, 3, size=H.n).astype(np.uint32)
    for u in range(H.n):
        for t in range(3):
            if t != part[u]:
                assert orc.graph_gain(H, adj, adjw, part, u, t) == bf.move_delta(H, part, u, t)


def _moves(rs, n, k, part, count, noop=2):
    us = rs.choice(n, size=count, replace=False).astype(np.uint32)
    ts = np.array([(int(part[u]) + 1 + rs.randint(k - 1)) % k for u in us], np.uint32)
    ts[:noop] = part[us[:noop]]  # moves to the node's own block
    return us, ts


@pytest.mark.parametrize("seed", range(8))
def test_graph_gain_table_is_w_u_vi(orc, seed):
    h, edges = random_graph(seed)
    rs = np.random.RandomState(300 + seed)
    for k in (2, 3, 6):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        om = orc.graph_gain_table(h, k, part)
        # each entry from its definition over the edge list
        want = np.zeros((h.n, k), np.int64)
        for (a, b), w in zip(edges, h.nwgt):
            want[a, part[b]] += int(w)
            want[b, part[a]] += int(w)
        assert np.array_equal(om, want)
        # gain = w(u, V_t) - w(u, V_Pi[u]) = the objective decrease by brute force
        for u in range(h.n):
            for t in range(k):
                if t != part[u]:
                    assert om[u, t] - om[u, part[u]] == bf.move_delta(h, part, u, t), (u, t)
    assert orc.graph_gain_table(W.from_nets(4, [[0, 1], [1, 2, 3]]), 2, np.zeros(4, np.uint32)) is None


@pytest.mark.parametrize("seed", range(8))
def test_graph_table_update_and_attributed_gains(orc, seed):
    h, edges = random_graph(seed, n=16, m=40)
    rs = np.random.RandomState(400 + seed)
    for k in (2, 4):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        us, ts = _moves(rs, h.n, k, part, 9)
        om0 = orc.graph_gain_table(h, k, part)
        new, g, om = orc.graph_moves(h, k, part, us, ts, om0)
        want_part = part.copy()
        want_part[us] = ts
        assert np.array_equal(new, want_part)
        # the updated table is the table of the new partition
        assert np.array_equal(om, orc.graph_gain_table(h, k, new))
        # attributed gains: the objective decrease of each move made in order
        moves = list(zip(us.tolist(), ts.tolist()))
        assert g.tolist() == bf.sequence_gains(h, part, moves)
        assert int(g.sum()) == bf.objective(h, part) - bf.objective(h, new)
        assert g.tolist() == orc.gain_recalc(h, k, part, us, ts).tolist()


def test_graph_moves_rejects_invalid(orc):
    h, _ = random_graph(1)
    part = np.zeros(h.n, np.uint32)
    for us, ts in (([1, 2, 1], [1, 1, 1]), ([h.n], [1]), ([3], [2])):
        with pytest.raises(ValueError):
            orc.graph_moves(h, 2, part, us, ts)
