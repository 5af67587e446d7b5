"""Pins of the CPU oracle: published values, definitions by brute force,
closed-form special cases and hand-derived fixtures.  No GPU needed."""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
from paper_2303_17679_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny(seed, n=9, m=8, smax=4, wmax=3, vmax=1, single=False):
    """Small random hypergraph; sizes 1..smax (or 2..smax), weights 1..wmax."""
    rs = np.random.RandomState(seed)
    nets = []
    for _ in range(m):
        s = rs.randint(1 if single else 2, smax + 1)
        nets.append(sorted(rs.choice(n, size=min(s, n), replace=False).tolist()))
    return W.from_nets(n, nets, vwgt=rs.randint(1, vmax + 1, size=n), nwgt=rs.randint(1, wmax + 1, size=m))


def test_splitmix64_published_values(orc):
    # SplitMix64 (Steele, Lea, Flood 2014) seeded with 1234567: the first five
    # outputs of its reference implementation; output i = finalizer(seed + i*golden).
    golden = 0x9E3779B97F4A7C15
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    got = [orc.mix64((1234567 + i * golden) % 2**64) for i in range(1, 6)]
    assert got == expect


def test_generator_rng_matches_published_splitmix(orc):
    # the input generators' counter RNG uses the same published finalizer
    z = np.array([(1234567 + i * 0x9E3779B97F4A7C15) % 2**64 for i in range(1, 6)], dtype=np.uint64)
    assert [int(x) for x in W._mix64(z)] == [orc.mix64(int(x)) for x in z]


def test_lmax_exact_rational(orc):
    # L_max = (1+eps) ceil(c(V)/k), eps = 3/100 (Sec. 2): largest integer <= the real bound
    for Wt, k in [(10000, 2), (4096000, 64), (3, 2), (1000001, 8), (7, 3)]:
        per = -(-Wt // k)
        bound = 1.03 * per
        lm = orc.lmax(Wt, k)
        assert lm <= bound + 1e-9 and lm + 1 > bound - 1e-9
    assert orc.lmax(10000, 2) == 5150
    assert orc.lmax(4096000, 64) == 65920


def test_golden_small6(orc):
    d = json.load(open(os.path.join(GOLD, "small6.json")))
    h = W.from_nets(d["n"], d["nets"], nwgt=d["nwgt"])
    part = np.array(d["part"], np.uint32)
    f, bw = orc.objective(h, d["k"], part)
    assert f == d["objective"]
    for u, t, g in d["gains"]:
        assert orc.gain(h, part, u, t) == g
    # rating from the first coarsening sub-round state (all singletons)
    u = d["rating_u"]
    rep = np.arange(d["n"], dtype=np.uint32)
    R = bf.rating(h, rep, u)
    assert {str(c): v for c, v in R.items()} == d["rating_all_singletons"]
    cid, H = orc.contract(h, np.array(d["contract_rep"], np.uint32))
    assert cid.tolist() == d["contract_cid"]
    assert [H.pins[H.pin_off[e]:H.pin_off[e + 1]].tolist() for e in range(H.m)] == d["contract_nets"]
    assert H.nwgt.tolist() == d["contract_nwgt"]
    assert H.vwgt.tolist() == d["contract_vwgt"]
    assert [H.inc[H.inc_off[v]:H.inc_off[v + 1]].tolist() for v in range(H.n)] == d["contract_inc"]


def test_golden_conflict_swap(orc):
    d = json.load(open(os.path.join(GOLD, "conflict3.json")))
    h = W.from_nets(d["n"], d["nets"], nwgt=d["nwgt"])
    part = np.array(d["part_in"], np.uint32)
    for u, t, g in d["gains"]:
        assert orc.gain(h, part, u, t) == g
    assert orc.lmax(3, 2, tuple(d["eps"])) == d["lmax"]
    assert orc.objective(h, 2, part)[0] == d["f_in"]
    P = orc.params(2, eps=tuple(d["eps"]), lp_rounds=d["lp_rounds"], lp_subrounds=d["lp_subrounds"])
    out, f, bw, rounds, moves = orc.refine_lp(h, P, 0, part)
    assert out.tolist() == d["part_out"] and f == d["f_out"] and moves == 2
    P = orc.params(2, eps=tuple(d["tight_eps"]), lp_rounds=1, lp_subrounds=1)
    out, f, bw, rounds, moves = orc.refine_lp(h, P, 0, part)
    assert out.tolist() == d["tight_part_out"] and f == d["tight_f_out"] and moves == 1


@pytest.mark.parametrize("seed", range(12))
def test_objective_bruteforce(orc, seed):
    h = tiny(seed, single=True)
    rs = np.random.RandomState(100 + seed)
    for k in (2, 3, 5):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        f, bw = orc.objective(h, k, part)
        assert f == bf.objective(h, part)
        assert bw.tolist() == [int(h.vwgt[part == b].sum()) for b in range(k)]
        if k == 2:  # for bipartitions the connectivity metric equals the cut-net metric
            assert f == bf.cut_net(h, part)


def test_objective_graph_is_edge_cut(orc):
    rs = np.random.RandomState(5)
    edges = set()
    while len(edges) < 40:
        a, b = sorted(rs.choice(20, 2, replace=False).tolist())
        edges.add((a, b))
    edges = sorted(edges)
    wts = rs.randint(1, 5, size=len(edges))
    h = W.from_nets(20, edges, nwgt=wts)
    part = rs.randint(0, 6, size=20).astype(np.uint32)
    cut = sum(int(w) for (a, b), w in zip(edges, wts) if part[a] != part[b])
    assert orc.objective(h, 6, part)[0] == cut


@pytest.mark.parametrize("seed", range(10))
def test_gain_is_objective_delta(orc, seed):
    # g_u(t) = f(Pi) - f(Pi[u -> t]) for every node and every other block
    h = tiny(seed, n=8, m=9, single=True)
    rs = np.random.RandomState(200 + seed)
    k = 4
    part = rs.randint(0, k, size=h.n).astype(np.uint32)
    for u in range(h.n):
        for t in range(k):
            if t != part[u]:
                assert orc.gain(h, part, u, t) == bf.move_delta(h, part, u, t), (u, t)


def random_clustering(h, rs, frac=0.4):
    """A valid clustering state: representatives own their clusters."""
    n = h.n
    rep = np.arange(n, dtype=np.uint32)
    reps = [v for v in range(n) if rs.rand() > frac] or [0]
    for v in range(n):
        if v not in reps:
            rep[v] = reps[rs.randint(len(reps))]
    cw = np.zeros(n, np.int64)
    cs = np.zeros(n, np.uint32)
    for v in range(n):
        cw[rep[v]] += h.vwgt[v]
        cs[rep[v]] += 1
    for v in range(n):
        if rep[v] != v:
            cw[v], cs[v] = h.vwgt[v], 1  # stale entries of non-representatives are never read
    return rep, cw, cs


@pytest.mark.parametrize("seed", range(12))
def test_rating_and_target_bruteforce(orc, seed):
    h = tiny(seed, n=12, m=14, smax=5, wmax=4, vmax=2)
    rs = np.random.RandomState(300 + seed)
    rep, cw, cs = random_clustering(h, rs)
    Wt = int(h.vwgt.sum())
    for k, lf in ((2, 1), (2, 3)):  # small limit factors so the cluster cap binds
        P = orc.params(k, seed=seed, limit_factor=lf, coarsen_subrounds=2)
        for r in range(2):
            target, nc = orc.rate_subround(h, P, 0, r, rep, cw, cs)
            cand = [u for u in range(h.n) if rep[u] == u and cs[u] == 1
                    and bf.H(seed, 1, 0, 0, u) % 2 == r]
            assert nc == len(cand)
            for u in range(h.n):
                if u not in cand:
                    assert target[u] == orc.NONE
                    continue
                R = bf.rating(h, rep, u)
                ok = [C for C in R if lf * k * (int(h.vwgt[u]) + int(cw[C])) <= Wt and C not in cand]
                if not ok:
                    assert target[u] == orc.NONE
                    continue
                best = min(ok, key=lambda C: (-R[C], bf.H(seed, 2, 0, 0, C), C))
                assert target[u] == best, (u, R, ok)


@pytest.mark.parametrize("seed", range(10))
def test_approval_longest_prefix(orc, seed):
    h = tiny(seed, n=14, m=16, smax=5, vmax=4)
    rs = np.random.RandomState(400 + seed)
    rep, cw, cs = random_clustering(h, rs, frac=0.3)
    P = orc.params(2, seed=seed, limit_factor=1, coarsen_subrounds=1)
    target, _ = orc.rate_subround(h, P, 0, 0, rep, cw, cs)
    rep2, cw2, cs2 = rep.copy(), cw.copy(), cs.copy()
    napp = orc.approve_apply(h, P, target, rep2, cw2, cs2)
    Wt = int(h.vwgt.sum())
    groups = {}
    for u in range(h.n):
        if target[u] != orc.NONE:
            groups.setdefault(int(target[u]), []).append(u)
    total = 0
    for C, us in groups.items():
        us.sort(key=lambda u: (int(h.vwgt[u]), u))
        # longest prefix that keeps 2 * (c(C) + prefix) <= c(V), by enumeration
        best = 0
        for L in range(len(us) + 1):
            if 2 * (int(cw[C]) + sum(int(h.vwgt[u]) for u in us[:L])) <= Wt:
                best = L
        for i, u in enumerate(us):
            assert (rep2[u] == C) == (i < best)
        total += best
        assert cw2[C] == cw[C] + sum(int(h.vwgt[u]) for u in us[:best])
    assert napp == total


@pytest.mark.parametrize("seed", range(15))
def test_contraction_sets_and_projection_invariant(orc, seed):
    h = tiny(seed, n=12, m=20, smax=5, wmax=5, vmax=3, single=True)
    rs = np.random.RandomState(500 + seed)
    rep, _, _ = random_clustering(h, rs, frac=0.5)
    cid, H = orc.contract(h, rep)
    reps = sorted(set(int(x) for x in rep))
    assert H.n == len(reps)
    assert cid.tolist() == [reps.index(int(rep[v])) for v in range(h.n)]
    # coarse nets by sets, named by representative
    expect = bf.contract_sets(h, rep)
    got = {}
    for e in range(H.m):
        s = frozenset(reps[int(x)] for x in H.pins[H.pin_off[e]:H.pin_off[e + 1]])
        assert s not in got  # identical nets merged
        got[s] = int(H.nwgt[e])
    assert got == expect
    # kept net order: ascending smallest fine net ID of each group
    first = {}
    for e, pins in enumerate(bf.nets_of(h)):
        s = frozenset(int(rep[v]) for v in pins)
        if len(s) >= 2 and s not in first:
            first[s] = e
    order = sorted(first, key=lambda s: first[s])
    assert [frozenset(reps[int(x)] for x in H.pins[H.pin_off[e]:H.pin_off[e + 1]]) for e in range(H.m)] == order
    # pins ascending, incidence = exact transpose with ascending nets
    for e in range(H.m):
        p = H.pins[H.pin_off[e]:H.pin_off[e + 1]]
        assert np.all(np.diff(p.astype(np.int64)) > 0)
    tr = {v: [] for v in range(H.n)}
    for e in range(H.m):
        for x in H.pins[H.pin_off[e]:H.pin_off[e + 1]]:
            tr[int(x)].append(e)
    assert all(H.inc[H.inc_off[v]:H.inc_off[v + 1]].tolist() == tr[v] for v in range(H.n))
    # weights preserved; objective invariant under projection for random partitions
    assert int(H.vwgt.sum()) == int(h.vwgt.sum())
    for k in (2, 3, 4):
        cp = rs.randint(0, k, size=H.n).astype(np.uint32)
        fp = orc.project(cid, cp)
        fc, bwc = orc.objective(H, k, cp)
        ff, bwf = orc.objective(h, k, fp)
        assert fc == ff == bf.objective(h, fp)
        assert bwc.tolist() == bwf.tolist()


@pytest.mark.parametrize("seed", range(300))
def test_pair_selection_last_feasible_on_merge_path(orc, seed):
    rs = np.random.RandomState(seed)
    la, lb = rs.randint(0, 7), rs.randint(0, 7)
    ca = rs.randint(1, 5, size=la)
    cb = rs.randint(1, 5, size=lb)
    bs, bt = rs.randint(-2, 6), rs.randint(-2, 6)
    found, i, j = orc.select_pair(ca, cb, bs, bt)
    states = bf.merge_path_states(ca.tolist(), cb.tolist())
    feas = [(a, b) for a, b in states if -bs <= int(ca[:a].sum()) - int(cb[:b].sum()) <= bt]
    if feas:
        assert found and (i, j) == feas[-1]
    else:
        assert not found and (i, j) == (0, 0)


def test_pair_selection_k2_is_paper_rule(orc):
    # k = 2: beta_b = L_max - c(V_b), i.e. the paper's feasibility test exactly
    rs = np.random.RandomState(7)
    for _ in range(200):
        ca = rs.randint(1, 4, size=rs.randint(0, 6))
        cb = rs.randint(1, 4, size=rs.randint(0, 6))
        lmax, ws, wt = 20, rs.randint(10, 22), rs.randint(10, 22)
        found, i, j = orc.select_pair(ca, cb, lmax - ws, lmax - wt)
        if found:
            x = int(ca[:i].sum()) - int(cb[:j].sum())
            assert ws - x <= lmax and wt + x <= lmax


@pytest.mark.parametrize("seed", range(8))
def test_greedy_ip_bounds_and_bfs_order(orc, seed):
    h = tiny(seed, n=30, m=25, smax=4, vmax=3, single=True)
    for k in (2, 3, 7):
        part = orc.greedy_ip(h, k)
        Wt = int(h.vwgt.sum())
        T = -(-Wt // k)
        cmax = int(h.vwgt.max())
        bw = [int(h.vwgt[part == b].sum()) for b in range(k)]
        assert all(x <= T + cmax - 1 for x in bw)
        # blocks are consecutive runs of one BFS order, filled in increasing block order
        nonempty = [b for b in range(k) if bw[b] > 0]
        assert nonempty == list(range(len(nonempty)))
        assert all(bw[b] >= T for b in nonempty[:-1] if b < k - 1)


@pytest.mark.parametrize("seed", range(6))
def test_lp_result_balanced_consistent(orc, seed):
    h = W.random_uniform(400, 400, 2, 6, seed=seed)
    for k in (2, 4):
        P = orc.params(k, seed=seed)
        part = orc.greedy_ip(h, k)
        out, f, bw, rounds, moves = orc.refine_lp(h, P, 0, part)
        lm = orc.lmax(int(h.vwgt.sum()), k)
        assert bw.max() <= lm
        assert f == bf.objective(h, out)
        assert bw.tolist() == [int(h.vwgt[out == b].sum()) for b in range(k)]
        out2, f2, *_ = orc.refine_lp(h, P, 0, part)
        assert np.array_equal(out, out2) and f == f2  # external determinism


def test_lp_independent_moves_sum_of_gains(orc):
    # disjoint components, each a 3-pin net with exactly one profitable node
    # (the lone pin in the minority block): the moves cannot interact, so the
    # objective drops by exactly the sum of their snapshot gains (Sec. 6 gain)
    nets, wts, part = [], [], []
    comps = 8
    for c in range(comps):
        nets.append([3 * c, 3 * c + 1, 3 * c + 2])
        wts.append(1 + c)
        part += [0, 0, 1] if c % 2 == 0 else [1, 1, 0]
    h = W.from_nets(3 * comps, nets, nwgt=wts)
    part = np.array(part, np.uint32)
    k = 2
    gains = {u: orc.gain(h, part, u, 1 - int(part[u])) for u in range(h.n)}
    assert sum(g > 0 for g in gains.values()) == comps
    P = orc.params(k, eps=(99, 100), lp_rounds=1, lp_subrounds=1)
    out, f, bw, rounds, moves = orc.refine_lp(h, P, 0, part)
    moved = [u for u in range(h.n) if out[u] != part[u]]
    assert len(moved) == comps and all(gains[u] > 0 for u in moved)
    assert bf.objective(h, part) - f == sum(gains[u] for u in moved) == sum(wts)


@pytest.mark.parametrize("name,k", [("random10k", 2), ("stencil24", 64)])
def test_partition_end_to_end_valid(orc, name, k):
    h, _ = W.workload(name)
    P = orc.params(k, seed=11)
    part, f, L = orc.partition(h, P)
    assert part.max() < k
    Wt = int(h.vwgt.sum())
    bw = np.bincount(part, weights=h.vwgt, minlength=k)
    assert bw.max() <= orc.lmax(Wt, k)
    assert f == orc.objective(h, k, part)[0]
    part2, f2, L2 = orc.partition(h, P)
    assert np.array_equal(part, part2) and f == f2 and L == L2
    lv = orc.hierarchy(h, P)
    assert np.array_equal(lv[0]["part"], part) and lv[0]["f"] == f
    for l in range(len(lv) - 1):  # every contraction keeps c(V) and shrinks n by more than 1 %
        assert int(lv[l + 1]["h"].vwgt.sum()) == Wt
        assert 100 * (lv[l]["h"].n - lv[l + 1]["h"].n) > lv[l]["h"].n


def test_cluster_pass_cap_and_invariants(orc):
    h = W.random_uniform(3000, 3000, 2, 6, seed=4)
    P = orc.params(4, seed=2)
    rep, cnt, run = orc.cluster_pass(h, P, 0)
    assert np.all(rep[rep] == rep)  # representatives own their clusters
    assert cnt == int((rep == np.arange(h.n)).sum())
    cw = np.bincount(rep, weights=h.vwgt, minlength=h.n)
    Wt = int(h.vwgt.sum())
    assert all(160 * 4 * cw[c] <= Wt or cw[c] == h.vwgt[c] for c in range(h.n) if rep[c] == c)
    # a pass that ended early left fewer than n/2.5 clusters (the rule itself
    # is replayed sub-round by sub-round in test_oracle_rules)
    assert run == 3 or 5 * cnt < 2 * h.n


def bfs_order_reference(h):
    """The initial partition's order from its definition, in plain Python:
    breadth first from the smallest unvisited vertex, neighbours in ascending
    incident-net order and ascending pin order inside a net."""
    nets = bf.nets_of(h)
    inc = [[] for _ in range(h.n)]
    for e, pins in enumerate(nets):
        for v in pins:
            inc[v].append(e)
    seen, order = set(), []
    for start in range(h.n):
        if start in seen:
            continue
        seen.add(start)
        queue = [start]
        while queue:
            v = queue.pop(0)
            order.append(v)
            for e in sorted(inc[v]):
                for w in nets[e]:
                    if w not in seen:
                        seen.add(w)
                        queue.append(w)
    return order


@pytest.mark.parametrize("seed", range(8))
def test_greedy_ip_matches_definition(orc, seed):
    h = tiny(seed, n=40, m=30, smax=4, vmax=3, single=True)
    order = bfs_order_reference(h)
    for k in (2, 3, 6):
        T = -(-int(h.vwgt.sum()) // k)
        expect = [0] * h.n
        b, cb = 0, 0
        for v in order:
            expect[v] = b
            cb += int(h.vwgt[v])
            if cb >= T and b < k - 1:
                b, cb = b + 1, 0
        assert orc.greedy_ip(h, k).tolist() == expect


@pytest.mark.parametrize("seed", range(10))
def test_lp_proposals_bruteforce(orc, seed):
    # best move of every candidate: the largest positive objective decrease
    # among blocks that can take the node within L_max, ties to the smaller block
    h = tiny(seed, n=10, m=12, smax=4, wmax=4, vmax=2, single=True)
    rs = np.random.RandomState(900 + seed)
    k = 3
    part = rs.randint(0, k, size=h.n).astype(np.uint32)
    for eps in ((3, 100), (1, 2)):
        P = orc.params(k, eps=eps, seed=seed, lp_subrounds=2)
        Wt = int(h.vwgt.sum())
        lm = orc.lmax(Wt, k, eps)
        bw = [int(h.vwgt[part == b].sum()) for b in range(k)]
        for s in range(2):
            t, g = orc.lp_proposals(h, P, 0, 1, s, part)
            for u in range(h.n):
                if bf.H(seed, 3, 0, 1, u) % 2 != s:
                    assert t[u] == orc.NONE
                    continue
                best = None
                for tt in range(k):
                    if tt == part[u] or bw[tt] + int(h.vwgt[u]) > lm:
                        continue
                    d = bf.move_delta(h, part, u, tt)
                    if d > 0 and (best is None or d > best[0]):
                        best = (d, tt)
                if best is None:
                    assert t[u] == orc.NONE
                else:
                    assert (int(t[u]), int(g[u])) == (best[1], best[0])
