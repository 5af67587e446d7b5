"""Pins of the recursive-bipartitioning initial partition (Sec. 5, Eq. 1) in
the oracle: the bisection limits against Eq. 1's closed forms and the balance
lemma it serves, the subhypergraph against its definition, LP with per-block
limits against the uniform LP, the targeted greedy fill, and the recursion
replayed in Python from the oracle's bisections.  No GPU."""
from fractions import Fraction
import math

import numpy as np
import pytest

import bruteforce as bf
from paper_2303_17679_amd import workloads as W
from test_oracle import tiny


@pytest.mark.parametrize("W_,k", [(1000, 2), (4097, 2), (123457, 2), (10**6 + 3, 2)])
def test_top_bisection_limit_is_lmax(orc, W_, k):
    # for k' = k = 2, Eq. 1 gives eps' = eps: each side's limit is (1 + eps) ceil(W / 2)
    L, T = orc.rb_limits(W_, k, (3, 100), W_, k)
    assert T == [(W_ + 1) // 2, (W_ + 1) // 2]
    exact = math.floor(Fraction(103, 100) * T[0])
    assert L == [exact, exact]


@pytest.mark.parametrize("k", [3, 4, 8, 11, 64, 256])
def test_limits_compose_to_eps(orc, k):
    # the lemma behind Eq. 1: if every bisection on the path to a block uses
    # its side's limit in full (the worst case), the block still ends within
    # (1 + eps) c(V) / k -- eps' adapts to the weight the subproblem really got
    Wt = 3 * 5 * 7 * 1000 * k + 17
    Wsub, kk = Wt, k
    steps = 0
    while kk > 1:
        L, T = orc.rb_limits(Wt, k, (3, 100), Wsub, kk)
        assert T[0] == -(-Wsub * ((kk + 1) // 2) // kk) and L[0] >= T[0]
        Wsub, kk = L[0], (kk + 1) // 2
        steps += 1
    bound = Fraction(103, 100) * Fraction(Wt, k)
    assert Wsub <= bound + steps  # the ceilings of the targets add at most one unit per bisection
    assert Wsub >= bound * Fraction(99, 100)


def test_uneven_split_targets(orc):
    # k' = 5: side 0 gets 3 blocks, side 1 two; targets ceil(W k_i / 5)
    L, T = orc.rb_limits(1000, 5, (3, 100), 1000, 5)
    assert T == [600, 400]
    assert L[0] >= T[0] and L[1] >= T[1] and L[0] * 2 > L[1] * 3 - 3


@pytest.mark.parametrize("seed", range(8))
def test_subhypergraph_is_the_definition(orc, seed):
    h = tiny(seed, n=12, m=14, smax=5, wmax=4, vmax=3, single=True)
    rs = np.random.RandomState(seed)
    part = rs.randint(0, 2, size=h.n).astype(np.uint32)
    for side in (0, 1):
        S, vmap = orc.subhypergraph(h, part, side)
        keep = [v for v in range(h.n) if part[v] == side]
        assert vmap.tolist() == keep
        new = {v: i for i, v in enumerate(keep)}
        want = [(tuple(new[v] for v in pins if v in new), int(h.nwgt[e]))
                for e, pins in enumerate(bf.nets_of(h)) if any(v in new for v in pins)]
        got = [(tuple(S.pins[S.pin_off[e]:S.pin_off[e + 1]].tolist()), int(S.nwgt[e])) for e in range(S.m)]
        assert got == want
        assert S.vwgt.tolist() == [int(h.vwgt[v]) for v in keep]
        for i in range(S.n):
            assert S.inc[S.inc_off[i]:S.inc_off[i + 1]].tolist() == [e for e, (pins, _) in enumerate(want) if i in pins]


@pytest.mark.parametrize("name,k", [("random2k", 2), ("stencil16", 8), ("powerlaw20000", 4)])
def test_uniform_limits_are_the_plain_lp(orc, name, k):
    h = W.random_uniform(2000, 2000, 2, 8, seed=9, name=name) if name == "random2k" else W.workload(name)[0]
    P = orc.params(k, seed=2)
    part = orc.greedy_ip(h, k)
    L = orc.lmax(int(h.vwgt.sum()), k)
    a = orc.refine_lp(h, P, 0, part)
    b = orc.refine_lp_limits(h, P, 0, part, [L] * k)
    assert a[0].tolist() == b[0].tolist() and a[1] == b[1] and a[2].tolist() == b[2].tolist()
    assert a[3:] == b[3:]


@pytest.mark.parametrize("seed", range(6))
def test_per_block_limits_hold(orc, seed):
    h = W.random_uniform(600, 700, 2, 6, seed=seed, name="r")
    Wt = int(h.vwgt.sum())
    P = orc.params(2, seed=seed)
    T0 = Wt * 3 // 5
    part = orc.greedy_ip_targets(h, 2, [T0, Wt - T0])
    bw0 = [int(h.vwgt[part == b].sum()) for b in (0, 1)]
    L = [bw0[0] + 5, bw0[1] + 2]  # tight and uneven, feasible at the start
    out, f, bw, rounds, moves = orc.refine_lp_limits(h, P, 0, part, L)
    assert moves > 0 and bw[0] <= L[0] and bw[1] <= L[1]
    assert f == orc.objective(h, 2, out)[0]


def test_targeted_fill(orc):
    h = W.random_uniform(500, 500, 2, 6, seed=4, name="r")
    Wt = int(h.vwgt.sum())
    # uniform targets: the greedy initial partition
    assert orc.greedy_ip_targets(h, 2, [(Wt + 1) // 2] * 2).tolist() == orc.greedy_ip(h, 2).tolist()
    # block 0 grows with its target, and it is the shortest prefix of the order reaching it
    prev = set()
    for T0 in (50, 120, 250, 400):
        p = orc.greedy_ip_targets(h, 2, [T0, Wt])
        b0 = {v for v in range(h.n) if p[v] == 0}
        assert prev <= b0
        assert sum(int(h.vwgt[v]) for v in b0) >= T0
        prev = b0


def test_small_bisection_is_fill_plus_lp(orc):
    # at most 160 k = 320 vertices: no coarsening, so a bisection is the
    # targeted fill followed by LP with the side limits
    h = W.random_uniform(300, 320, 2, 6, seed=8, name="r")
    Wt = int(h.vwgt.sum())
    P = orc.params(5, seed=3)
    L, T = orc.rb_limits(Wt, 5, (3, 100), Wt, 5)
    got = orc.bisect(h, P, L, T)
    P2 = orc.params(2, seed=3)
    want = orc.refine_lp_limits(h, P2, 0, orc.greedy_ip_targets(h, 2, T), L)[0]
    assert got.tolist() == want.tolist()


def replay_rb(orc, h, P):
    """The recursion of Sec. 5 written out again from the oracle's pieces."""
    Wt, k = int(h.vwgt.sum()), P.k
    out = np.full(h.n, orc.NONE, np.uint32)

    def rec(H, vmap, kk, b0):
        if H.n == 0:
            return
        if kk == 1:
            out[vmap] = b0
            return
        L, T = orc.rb_limits(Wt, k, (P.eps_num, P.eps_den), int(H.vwgt.sum()), kk)
        bp = orc.bisect(H, P, L, T)
        for side, kb, bb in ((0, (kk + 1) // 2, b0), (1, kk // 2, b0 + (kk + 1) // 2)):
            S, smap = orc.subhypergraph(H, bp, side)
            rec(S, vmap[smap], kb, bb)

    rec(h, np.arange(h.n, dtype=np.uint32), k, 0)
    return out


@pytest.mark.parametrize("name,k", [("random2k", 3), ("random2k", 8), ("stencil16", 6), ("stencil24", 64),
                                    ("powerlaw20000", 7)])
def test_recursion_replayed(orc, name, k):
    h = W.random_uniform(2000, 2000, 2, 8, seed=9, name=name) if name == "random2k" else W.workload(name)[0]
    P = orc.params(k, seed=4)
    part = orc.rb_ip(h, P)
    assert part.tolist() == replay_rb(orc, h, P).tolist()
    assert sorted(set(part.tolist())) == list(range(k))


def test_a_full_block_takes_no_node(orc):
    # two clusters X = 0..99 and Y = 100..199 (nets inside each); ten Y nodes
    # start in block 0 and ten X nodes in block 1, and block 1 is at its
    # limit: the X nodes propose to go home to block 0, the Y nodes propose
    # nothing (block 1 cannot take them) although they would gain
    rs = np.random.RandomState(5)
    nets = [sorted(rs.choice(100, 4, replace=False).tolist()) for _ in range(300)]
    nets += [sorted((100 + rs.choice(100, 4, replace=False)).tolist()) for _ in range(300)]
    h = W.from_nets(200, nets)
    part = np.array([0] * 100 + [1] * 100, np.uint32)
    part[100:110] = 0
    part[:10] = 1
    Wt = int(h.vwgt.sum())
    bw1 = int(h.vwgt[part == 1].sum())
    P = orc.params(2, seed=1, lp_subrounds=1)
    t, g = orc.lp_proposals_limits(h, P, 0, 0, 0, part, [Wt, bw1])
    assert all(t[v] == 0 for v in range(10))  # the X nodes propose to go home
    assert all(t[v] == orc.NONE for v in range(100, 110))  # the Y nodes could gain, but block 1 is full
    t2, g2 = orc.lp_proposals_limits(h, P, 0, 0, 0, part, [Wt, Wt])
    assert all(t2[v] == 1 and g2[v] > 0 for v in range(100, 110))  # with room they do propose
    out, f, bw, rounds, moves = orc.refine_lp_limits(h, P, 0, part, [Wt, bw1])
    assert all(out[v] == 0 for v in range(10)) and bw[1] <= bw1


def test_bisections_ignore_communities(orc):
    # community detection runs on the input only; a bisection never runs it
    h = W.random_uniform(1500, 1500, 2, 6, seed=3, name="r")
    Wt = int(h.vwgt.sum())
    L, T = orc.rb_limits(Wt, 4, (3, 100), Wt, 4)
    a = orc.bisect(h, orc.params(4, seed=2), L, T)
    b = orc.bisect(h, orc.params(4, seed=2, community=True), L, T)
    assert a.tolist() == b.tolist()
