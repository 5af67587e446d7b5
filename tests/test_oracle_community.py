"""Pins of the community detection (Sec. 4.3, deterministic Louvain of
Sec. 11) and of the community-restricted clustering in the oracle: the
bipartite graph from its definition, every local-moving sub-round against
exact modularity (fractions, recomputed from scratch per candidate move), the
multilevel composition replayed in Python, and the restriction of ratings and
clusters to communities.  No GPU."""
import numpy as np
import pytest

import bruteforce as bf
from paper_2303_17679_amd import workloads as W
from test_oracle import tiny, random_clustering


def graph_edges(g):
    return [(int(g.pins[g.pin_off[e]]), int(g.pins[g.pin_off[e] + 1]), int(g.nwgt[e])) for e in range(g.m)]


@pytest.mark.parametrize("seed", range(8))
def test_bipartite_graph_from_definition(orc, seed):
    h = tiny(seed, n=10, m=9, smax=5, wmax=4, single=True)
    g = orc.bipartite(h)
    assert (g.n, g.m) == (h.n + h.m, h.p)
    want = bf.bipartite_edges(h)
    assert graph_edges(g) == [(a, b, w) for a, b, w in want]
    # incidence: every node lists exactly its edges, ascending
    for x in range(g.n):
        lst = g.inc[g.inc_off[x]:g.inc_off[x + 1]].tolist()
        assert lst == [j for j, (a, b, _) in enumerate(want) if x in (a, b)]
    # volumes: sum of incident edge weights
    vol = np.zeros(g.n, np.int64)
    for a, b, w in want:
        vol[a] += w
        vol[b] += w
    assert g.vwgt.tolist() == vol.tolist()


def random_weighted_graph(seed, n=12, m=24):
    rs = np.random.RandomState(seed)
    edges = [tuple(sorted(rs.choice(n, 2, replace=False).tolist())) for _ in range(m)]
    return W.from_nets(n, [list(e) for e in edges], nwgt=rs.randint(1, 5, size=m))


@pytest.mark.parametrize("kind,seed", [("graph", s) for s in range(6)] + [("bipartite", s) for s in range(4)])
def test_local_moving_subrounds_raise_modularity_exactly(orc, kind, seed):
    if kind == "graph":
        g = random_weighted_graph(seed)
        # vwgt must be the volumes for the local moving
        vol = np.zeros(g.n, np.int64)
        for a, b, w in graph_edges(g):
            vol[a] += w
            vol[b] += w
        g.vwgt = vol.astype(np.int32)
    else:
        g = orc.bipartite(tiny(20 + seed, n=8, m=7, smax=4, wmax=3))
    edges = graph_edges(g)
    level = seed % 3
    comm = np.arange(g.n, dtype=np.uint32)
    cvol = g.vwgt.astype(np.int64).copy()
    want = list(range(g.n))
    for r in range(3):
        for s in range(5):
            mv, comm, cvol = orc.louvain_subround(g, seed, level, r, s, comm, cvol)
            want, mv_b = bf.louvain_subround(edges, g.n, want, seed, level, r, s)
            assert comm.tolist() == want, (r, s)
            assert mv == mv_b
            # community volumes stay the sums of their members' volumes
            vol = {}
            for x in range(g.n):
                vol[int(comm[x])] = vol.get(int(comm[x]), 0) + int(g.vwgt[x])
            for c, v in vol.items():
                assert cvol[c] == v


def test_two_cliques_give_two_communities(orc):
    # two 6-cliques joined by one edge: the local moving ends with each clique
    # a community, the best modularity of this graph
    edges = [(a, b) for a in range(6) for b in range(a + 1, 6)]
    edges += [(a + 6, b + 6) for a, b in edges] + [(5, 6)]
    g = W.from_nets(12, [list(e) for e in edges])
    g.vwgt = np.array([sum(1 for e in edges if x in e) for x in range(12)], np.int32)
    comm, mv, rounds = orc.louvain_level(g, 3, 0)
    groups = {int(comm[x]) for x in range(6)}, {int(comm[x]) for x in range(6, 12)}
    assert len(groups[0]) == 1 and len(groups[1]) == 1 and groups[0] != groups[1]
    q = bf.modularity([(a, b, 1) for a, b in edges], comm.tolist())
    from fractions import Fraction
    M = len(edges)
    vol0 = sum(int(g.vwgt[x]) for x in range(6))
    assert q == 2 * (Fraction(15, M) - Fraction(vol0, 2 * M) ** 2)


def replay_communities(orc, h, seed):
    """R18 written out again: levels of local moving, contraction of every
    community into its smallest node, composition of the node maps."""
    g = orc.bipartite(h)
    N = g.n
    node = np.arange(N, dtype=np.uint32)
    levels = 0
    for level in range(16):
        comm, mv, _ = orc.louvain_level(g, seed, level)
        if mv == 0:
            break
        first = {}
        for x in range(g.n):
            first.setdefault(int(comm[x]), x)
        rep = np.array([first[int(comm[x])] for x in range(g.n)], np.uint32)
        cid, g2 = orc.contract(g, rep)
        # the coarse graph: volumes add up, edges between communities merged
        want = {}
        for a, b, w in graph_edges(g):
            ca, cb = int(cid[a]), int(cid[b])
            if ca != cb:
                key = (min(ca, cb), max(ca, cb))
                want[key] = want.get(key, 0) + w
        assert {(a, b): w for a, b, w in graph_edges(g2)} == want
        assert g2.vwgt.tolist() == np.bincount(cid, weights=g.vwgt, minlength=g2.n).astype(int).tolist()
        node = cid[node]
        levels += 1
        shrunk = g2.n < g.n
        g = g2
        if not shrunk:
            break
    return node[:h.n], levels


@pytest.mark.parametrize("seed", range(6))
def test_communities_are_the_replayed_levels(orc, seed):
    h = W.random_uniform(300, 260, 2, 5, seed=seed, name="c")
    comm, levels = orc.communities(h, seed)
    want, lv = replay_communities(orc, h, seed)
    assert levels == lv and levels >= 1
    assert comm.tolist() == want.tolist()


def test_communities_never_span_components(orc):
    a = W.random_uniform(200, 180, 2, 5, seed=1, name="a")
    nets = [a.pins[a.pin_off[e]:a.pin_off[e + 1]].tolist() for e in range(a.m)]
    nets += [[v + 200 for v in net] for net in nets]
    h = W.from_nets(400, nets)
    comm, _ = orc.communities(h, 7)
    assert not (set(comm[:200].tolist()) & set(comm[200:].tolist()))


def test_bipartite_volume_bound(orc):
    # a total volume of 2^31 or more is rejected
    h = W.from_nets(3, [[0, 1, 2]], nwgt=[1 << 29])
    assert orc.bipartite(h) is None
    with pytest.raises(ValueError):
        orc.communities(h)


@pytest.mark.parametrize("seed", range(10))
def test_restricted_rating_bruteforce(orc, seed):
    h = tiny(seed, n=12, m=14, smax=5, wmax=4, vmax=2)
    rs = np.random.RandomState(500 + seed)
    rep, cw, cs = random_clustering(h, rs)
    comm = rs.randint(0, 3, size=h.n).astype(np.uint32)
    for v in range(h.n):  # a cluster lies in one community
        comm[v] = comm[rep[v]]
    Wt = int(h.vwgt.sum())
    P = orc.params(2, seed=seed, limit_factor=3, coarsen_subrounds=2)
    for r in range(2):
        target, nc = orc.rate_subround_c(h, P, 0, r, rep, cw, cs, comm)
        cand = [u for u in range(h.n) if rep[u] == u and cs[u] == 1 and bf.H(seed, 1, 0, 0, u) % 2 == r]
        for u in range(h.n):
            if u not in cand:
                assert target[u] == orc.NONE
                continue
            R = bf.rating(h, rep, u)
            ok = [C for C in R if 3 * 2 * (int(h.vwgt[u]) + int(cw[C])) <= Wt and C not in cand
                  and comm[C] == comm[u]]
            best = min(ok, key=lambda C: (-R[C], bf.H(seed, 2, 0, 0, C), C)) if ok else orc.NONE
            assert target[u] == best
        # one community for all: the unrestricted rating
        t0, _ = orc.rate_subround(h, P, 0, r, rep, cw, cs)
        t1, _ = orc.rate_subround_c(h, P, 0, r, rep, cw, cs, np.zeros(h.n, np.uint32))
        assert t0.tolist() == t1.tolist()


@pytest.mark.parametrize("name,k,seed", [("random2k", 2, 1), ("stencil16", 8, 2), ("powerlaw20000", 4, 3)])
def test_community_partition_keeps_clusters_in_communities(orc, name, k, seed):
    h = W.random_uniform(2000, 2000, 2, 8, seed=9, name=name) if name == "random2k" else W.workload(name)[0]
    P = orc.params(k, seed=seed, community=True)
    lv = orc.hierarchy(h, P)
    assert "comm" in lv[0]
    comm0, _ = orc.communities(h, seed)
    assert lv[0]["comm"].tolist() == comm0.tolist()
    for L in lv:
        if "rep" in L:
            assert np.array_equal(L["comm"][L["rep"]], L["comm"])
    part, f, nl = orc.partition(h, P)
    assert f == lv[0]["f"] and nl == len(lv) - 1
    assert part.tolist() == lv[0]["part"].tolist()


def replay_level(edges, n_nodes, seed, level):
    """Local moving of one level from singletons, from the definition: rounds
    of five sub-rounds until a round moves nothing, at most five rounds."""
    comm = list(range(n_nodes))
    total, rounds = 0, 0
    while rounds < 5:
        mv = 0
        for s in range(5):
            comm, m = bf.louvain_subround(edges, n_nodes, comm, seed, level, rounds, s)
            mv += m
        rounds += 1
        total += mv
        if mv == 0:
            break
    return comm, total, rounds


def test_level_rounds_end_at_a_round_without_moves(orc):
    early = 0
    for seed in range(8):
        g = orc.bipartite(tiny(40 + seed, n=8, m=6, smax=4, wmax=3))
        comm, mv, rounds = orc.louvain_level(g, seed, 1)
        want, mv_b, rounds_b = replay_level(graph_edges(g), g.n, seed, 1)
        assert (comm.tolist(), mv, rounds) == (want, mv_b, rounds_b), seed
        early += rounds_b < 5
    assert early >= 3  # most of these settle: the stop rule is what ends them


def test_levels_stop_when_a_contraction_does_not_shrink(orc):
    # one vertex in one single-pin net: G_x is a single edge.  With seed 4556
    # both nodes share a sub-round in all five rounds of level 0, so they
    # swap communities every round (synchronous moves) and end apart: the
    # contraction does not shrink the graph and the levels stop there (with
    # seed 4556 they would merge on level 1, in different sub-rounds).
    h = W.from_nets(1, [[0]])
    g = orc.bipartite(h)
    comm, mv, rounds = orc.louvain_level(g, 4556, 0)
    assert (mv, rounds) == (10, 5) and comm.tolist() == [1, 0]
    c, levels = orc.communities(h, 4556)
    assert levels == 1
    assert replay_communities(orc, h, 4556)[1] == 1
