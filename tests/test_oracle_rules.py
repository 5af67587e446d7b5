"""Pins of the oracle's control rules: the seeded hash's tag layout, the pass
cut of a clustering pass (Sec. 4.1: a pass ends once the clustering leaves
fewer than n/2.5 clusters), the contraction stop when a pass removes at most
1 % of the vertices (Sec. 4.1), and the end of label propagation after a
round without moves.  Each test is built so that changing the rule in the
oracle (dropping it, moving its boundary, or swapping the hash fields) makes
it fail.  No GPU needed."""
import numpy as np
import pytest

import bruteforce as bf
from paper_2303_17679_amd import workloads as W


# ---------------------------------------------------------------------------
# Seeded hash
# ---------------------------------------------------------------------------
def test_python_hash_is_published_splitmix64():
    # the first outputs of SplitMix64 seeded with 1234567 (its reference
    # implementation): output i = finalizer(seed + i * golden gamma)
    golden = 0x9E3779B97F4A7C15
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    assert [bf.mix64(1234567 + i * golden) for i in range(1, 6)] == expect


def test_hash_tag_layout(orc):
    # every field set to values that differ from one another, so a swapped or
    # shifted field changes the result
    rs = np.random.RandomState(3)
    rows = [(0, 1, 0, 0, 0), (7, 2, 5, 0, 11), (7, 3, 5, 1, 11), (7, 3, 1, 5, 11),
            (2**64 - 1, 3, 255, 65535, 2**32 - 1), (123456789, 1, 3, 0, 99), (123456789, 1, 0, 3, 99),
            (5, 2, 9, 2, 9), (5, 2, 2, 9, 9)]
    for _ in range(200):
        rows.append((int(rs.randint(0, 2**31)) * 2**33 + int(rs.randint(0, 2**31)), int(rs.randint(1, 4)),
                     int(rs.randint(0, 256)), int(rs.randint(0, 256)), int(rs.randint(0, 2**32, dtype=np.uint64))))
    for seed, purpose, level, it, x in rows:
        assert orc.hash_(seed, purpose, level, it, x) == bf.H(seed, purpose, level, it, x), (seed, purpose, level, it, x)


def test_subround_membership_uses_the_tagged_hash(orc):
    # coarsening sub-round r of level l: the singletons u with
    # H(seed, 1, l, 0, u) mod S_c = r are exactly the candidates
    h = W.random_uniform(300, 300, 2, 5, seed=9)
    for level in (0, 3):
        P = orc.params(2, seed=21, coarsen_subrounds=3)
        rep = np.arange(h.n, dtype=np.uint32)
        cw = h.vwgt.astype(np.int64)
        cs = np.ones(h.n, np.uint32)
        for r in range(3):
            _, nc = orc.rate_subround(h, P, level, r, rep, cw, cs)
            assert nc == sum(1 for u in range(h.n) if bf.H(21, 1, level, 0, u) % 3 == r)


# ---------------------------------------------------------------------------
# Pass cut: replay the sub-rounds and apply the rule from its definition
# ---------------------------------------------------------------------------
def replay_pass(orc, h, P, level):
    """Runs a clustering pass sub-round by sub-round from the oracle's
    (separately pinned) rating and approval steps; stops after the first
    sub-round that leaves fewer than n/2.5 clusters.  Returns the state and
    the cluster count after every sub-round."""
    n = h.n
    rep = np.arange(n, dtype=np.uint32)
    cw = h.vwgt.astype(np.int64)
    cs = np.ones(n, np.uint32)
    cnt = n
    counts = []
    for r in range(P.coarsen_subrounds):
        target, _ = orc.rate_subround(h, P, level, r, rep, cw, cs)
        cnt -= orc.approve_apply(h, P, target, rep, cw, cs)
        counts.append(cnt)
        if cnt < n / 2.5:
            break
    return rep, cnt, counts


def _pass_cases():
    cases = []
    for seed in range(60):
        rs = np.random.RandomState(seed)
        n = int(rs.randint(6, 40))
        m = int(rs.randint(n // 2, 2 * n))
        h = W.random_uniform(n, m, 2, int(rs.randint(2, 6)), seed=seed)
        for sc in (2, 3, 4):
            cases.append((h, sc, seed))
    # stars and cliques: one sub-round can absorb most vertices
    for n in (10, 15, 20, 25):
        cases.append((W.from_nets(n, [[0, v] for v in range(1, n)]), 2, n))
        cases.append((W.from_nets(n, [list(range(n))]), 3, n))
    return cases


def test_pass_cut_stops_at_the_first_subround_below_n_over_2_5(orc):
    runs, boundary = {}, 0
    for h, sc, seed in _pass_cases():
        P = orc.params(2, seed=seed, limit_factor=1, coarsen_subrounds=sc)
        rep_x, cnt_x, counts = replay_pass(orc, h, P, 0)
        rep, cnt, run = orc.cluster_pass(h, P, 0)
        assert run == len(counts), (seed, sc, counts)
        assert cnt == cnt_x and np.array_equal(rep, rep_x)
        early = run < sc
        runs[early] = runs.get(early, 0) + 1
        boundary += sum(1 for c in counts[:-1] if 5 * c == 2 * h.n)  # exactly n/2.5: not below, continue
    # the case set covers both outcomes and the equality boundary
    assert runs.get(True, 0) >= 5 and runs.get(False, 0) >= 5, runs
    assert boundary >= 1


def equality_case():
    """n = 10 and exactly four clusters left after the first sub-round: 4 is
    not below 10/2.5, so the pass must go on to the next sub-round.  Built
    from the hash: the six candidates of sub-round 0 are joined, three each,
    onto two vertices of sub-round 1 through 2-pin nets; the other two
    vertices of sub-round 1 share a net."""
    n, sc = 10, 2
    for seed in range(2000):
        sub = [bf.H(seed, 1, 0, 0, u) % sc for u in range(n)]
        c0 = [u for u in range(n) if sub[u] == 0]
        c1 = [u for u in range(n) if sub[u] == 1]
        if len(c0) == 6 and len(c1) == 4:
            break
    else:
        raise AssertionError("no seed with a 6/4 split")
    nets = [[c0[i], c1[0]] for i in range(3)] + [[c0[i], c1[1]] for i in range(3, 6)] + [[c1[2], c1[3]]]
    return W.from_nets(n, nets), seed, sc, c0, c1


def test_pass_cut_equality_continues(orc):
    h, seed, sc, c0, c1 = equality_case()
    P = orc.params(2, seed=seed, limit_factor=1, coarsen_subrounds=sc)
    rep, cnt, run = orc.cluster_pass(h, P, 0)
    # sub-round 1's candidates are the unclustered singletons c1[2], c1[3]
    # (c1[0], c1[1] own clusters of four); both are candidates, so neither
    # may join the other (same-sub-round singletons are no targets)
    assert run == 2
    assert cnt == 4
    assert [int(rep[u]) for u in c0] == [c1[0]] * 3 + [c1[1]] * 3


# ---------------------------------------------------------------------------
# Contraction stops when a pass removes at most 1 % of the vertices
# ---------------------------------------------------------------------------
def _pairs_in_different_subrounds(seed, n, count, sc=3):
    sub = [bf.H(seed, 1, 0, 0, u) % sc for u in range(n)]
    pairs, used = [], set()
    for u in range(n):
        for v in range(u + 1, n):
            if len(pairs) == count:
                return pairs
            if u in used or v in used or sub[u] == sub[v]:
                continue
            pairs.append([u, v])
            used.update((u, v))
    return pairs


@pytest.mark.parametrize("n,joins,contracts", [(100, 1, False), (100, 2, True), (200, 2, False), (200, 3, True)])
def test_one_percent_rule_boundary(orc, n, joins, contracts):
    # disjoint 2-pin nets whose two pins fall in different coarsening
    # sub-rounds: each net gives exactly one join, so the pass removes
    # exactly `joins` of n vertices.  100 * removed <= n stops coarsening.
    seed = 5
    nets = _pairs_in_different_subrounds(seed, n, joins)
    assert len(nets) == joins
    h = W.from_nets(n, nets)
    P = orc.params(2, seed=seed, limit_factor=1)
    rep, cnt, run = orc.cluster_pass(h, P, 0)
    assert n - cnt == joins
    part, f, levels = orc.partition(h, P)
    assert (levels >= 1) == contracts
    lv = orc.hierarchy(h, P)
    assert (len(lv) >= 2) == contracts


# ---------------------------------------------------------------------------
# LP ends after a round without moves
# ---------------------------------------------------------------------------
def swap_instance():
    """k = 3, unit weights, 30 vertices, eps = 1/10: c(V) = 30, L_max = 11,
    every block weighs 10, so every pair budget floor((11 - 10)/2) is 0.
    Vertex a = 0 (block 0) gains 5 by moving to block 1 (net {0, 2, 3}, pins
    2 and 3 in block 1); vertex b = 1 (block 1) gains 4 by moving to block 0
    (net {1, 4, 5}, pins 4 and 5 in block 0).  No other vertex has a positive
    gain.  Alone, either move makes x = 1 > 0 = beta and is rejected; in the
    same sub-round the walk reaches (1, 1) with x = 0 and swaps both."""
    n = 30
    nets = [[0, 2, 3], [1, 4, 5]]
    part = np.full(n, 2, np.uint32)
    part[[0, 4, 5] + list(range(6, 13))] = 0
    part[[1, 2, 3] + list(range(13, 20))] = 1
    h = W.from_nets(n, nets, nwgt=[5, 4])
    return h, part


def _seed_for(rounds_together):
    for seed in range(5000):
        together = [bf.H(seed, 3, 0, r, 0) % 2 == bf.H(seed, 3, 0, r, 1) % 2 for r in range(len(rounds_together))]
        if together == rounds_together:
            return seed
    raise AssertionError("no seed")


def test_swap_instance_gains(orc):
    h, part = swap_instance()
    assert np.bincount(part, minlength=3).tolist() == [10, 10, 10]
    assert orc.lmax(30, 3, (1, 10)) == 11
    assert orc.gain(h, part, 0, 1) == 5 and bf.move_delta(h, part, 0, 1) == 5
    assert orc.gain(h, part, 1, 0) == 4 and bf.move_delta(h, part, 1, 0) == 4
    for u in range(2, 30):
        assert all(bf.move_delta(h, part, u, t) <= 0 for t in range(3) if t != part[u])


def test_lp_round_without_moves_ends_lp(orc):
    # round 0 puts a and b into different sub-rounds: no move is feasible,
    # so LP ends there, although round 1 (a different grouping) would swap them
    h, part = swap_instance()
    seed = _seed_for([False, True])
    P = orc.params(3, eps=(1, 10), seed=seed, lp_rounds=5, lp_subrounds=2)
    out, f, bw, rounds, moves = orc.refine_lp(h, P, 0, part)
    assert rounds == 1 and moves == 0
    assert np.array_equal(out, part) and f == 9


def test_lp_swap_in_one_subround(orc):
    # round 0 groups a and b: the swap is applied (f 9 -> 0); round 1 has no
    # move left and ends LP
    h, part = swap_instance()
    seed = _seed_for([True])
    P = orc.params(3, eps=(1, 10), seed=seed, lp_rounds=5, lp_subrounds=2)
    out, f, bw, rounds, moves = orc.refine_lp(h, P, 0, part)
    expect = part.copy()
    expect[0], expect[1] = 1, 0
    assert rounds == 2 and moves == 2
    assert np.array_equal(out, expect) and f == 0 == bf.objective(h, expect)
