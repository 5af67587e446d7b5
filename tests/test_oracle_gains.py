"""Pins of the gain-table oracle (Sec. 6.2) and of the gains of a move
sequence (Sec. 6.3) against brute force from the definitions.  No GPU."""
import numpy as np
import pytest

import bruteforce as bf
from paper_2303_17679_amd import workloads as W
from test_oracle import tiny


def random_moves(rs, n, k, part, count):
    """`count` distinct nodes, each moved once to a block other than its own."""
    us = rs.choice(n, size=min(count, n), replace=False)
    ts = [(int(part[u]) + 1 + rs.randint(k - 1)) % k for u in us]
    return [int(u) for u in us], ts


@pytest.mark.parametrize("seed", range(12))
def test_gain_table_definition_and_move_deltas(orc, seed):
    h = tiny(seed, n=10, m=12, smax=5, wmax=4, single=True)
    rs = np.random.RandomState(1000 + seed)
    for k in (2, 3, 5):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        ben, pen = orc.gain_table(h, k, part)
        b_bf, p_bf = bf.gain_table(h, k, part)
        assert ben.tolist() == b_bf and pen.tolist() == p_bf
        for u in range(h.n):
            assert pen[u][part[u]] == 0  # u itself is in its block
            for t in range(k):
                if t != part[u]:  # g_u(t) = b(u) - p(u, t) = f(Pi) - f(Pi[u -> t])
                    assert ben[u] - pen[u][t] == bf.move_delta(h, part, u, t), (u, t)


@pytest.mark.parametrize("seed", range(12))
def test_update_rules_give_the_table_of_the_new_partition(orc, seed):
    # after all updates of a move set, every unmoved node has the right
    # benefit and every node the right penalties (Sec. 6.2 lemma); the moved
    # nodes' benefits are recomputed
    h = tiny(seed, n=12, m=14, smax=5, wmax=3, single=True)
    rs = np.random.RandomState(2000 + seed)
    for k in (2, 4):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        ben, pen = orc.gain_table(h, k, part)
        mu, mt = random_moves(rs, h.n, k, part, rs.randint(1, h.n))
        new_part, ben2, pen2 = orc.gain_table_moves(h, k, part, mu, mt, ben, pen)
        expect = part.copy()
        for u, t in zip(mu, mt):
            expect[u] = t
        assert np.array_equal(new_part, expect)
        b_bf, p_bf = bf.gain_table(h, k, expect)
        assert ben2.tolist() == b_bf and pen2.tolist() == p_bf


@pytest.mark.parametrize("seed", range(15))
def test_sequence_gains(orc, seed):
    h = tiny(seed, n=12, m=16, smax=6, wmax=5, single=True)
    rs = np.random.RandomState(3000 + seed)
    for k in (2, 3, 6):
        part = rs.randint(0, k, size=h.n).astype(np.uint32)
        mu, mt = random_moves(rs, h.n, k, part, rs.randint(1, h.n + 1))
        g = orc.gain_recalc(h, k, part, mu, mt)
        moves = list(zip(mu, mt))
        expect = bf.sequence_gains(h, part, moves)
        assert g.tolist() == expect
        # the paper's per-net recalculation gives the same gains
        assert bf.alg4_gains(h, part, moves) == expect
        # their sum is the objective change of the whole sequence
        final = part.copy()
        for u, t in moves:
            final[u] = t
        assert sum(expect) == bf.objective(h, part) - bf.objective(h, final)


def test_sequence_gains_order_matters(orc):
    # net {0, 1, 2} in blocks [0, 0, 1]: moving 0 then 1 to block 1 makes the
    # second move remove the net from the cut (+w); in the other order the
    # roles swap.  Hand-derived: w = 3, f goes 3 -> 3 -> 0.
    h = W.from_nets(3, [[0, 1, 2]], nwgt=[3])
    part = np.array([0, 0, 1], np.uint32)
    assert orc.gain_recalc(h, 2, part, [0, 1], [1, 1]).tolist() == [0, 3]
    assert orc.gain_recalc(h, 2, part, [1, 0], [1, 1]).tolist() == [0, 3]
    assert orc.gain_recalc(h, 2, part, [2, 0], [0, 1]).tolist() == [3, -3]
