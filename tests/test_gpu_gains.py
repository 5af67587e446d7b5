"""GPU parity of the gain table (Sec. 6.2), its update by a batch of moves and
the gains of a move sequence (Sec. 6.3) against the oracle, through the C ABI.
Partitions and moves come from the oracle's greedy partition and seeded
random draws."""
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def make(name):
    if name == "hugenets":
        rs = np.random.RandomState(17)
        n = 3000
        nets = [rs.choice(n, size=rs.randint(2, 7), replace=False) for _ in range(3000)]
        nets += [rs.choice(n, size=sz, replace=False) for sz in (40, 70, 500, 1500)]
        return W.from_nets(n, nets, nwgt=rs.randint(1, 4, size=len(nets)))
    if name == "random3k":
        return W.random_uniform(3000, 3500, 2, 12, seed=5, name=name)
    return W.workload(name)[0]


CASES = [("random3k", 2), ("random3k", 5), ("random3k", 33), ("stencil16", 8), ("stencil24", 64),
         ("powerlaw20000", 8), ("hugenets", 4), ("hugenets", 100), ("random3k", 256)]


def partitions(orc, h, k, rs):
    """A greedy (mostly uncut) partition and a uniformly random one."""
    yield "greedy", orc.greedy_ip(h, k)
    yield "random", rs.randint(0, k, size=h.n).astype(np.uint32)


def moves_of(rs, h, k, part, count, noop=0):
    us = rs.choice(h.n, size=min(count, h.n), replace=False)
    ts = np.array([(int(part[u]) + 1 + rs.randint(k - 1)) % k for u in us], np.uint32)
    if noop:  # some moves to the node's own block (no move)
        ts[:noop] = part[us[:noop]]
    return us.astype(np.uint32), ts


@pytest.mark.parametrize("name,k", CASES)
def test_gain_table_matches_oracle(hgp, orc, name, k):
    H = hgp
    h = make(name)
    G = H.Hypergraph.from_host(h)
    rs = np.random.RandomState(k)
    for kind, part in partitions(orc, h, k, rs):
        say(f"[gains] table {name} k={k} {kind}")
        ben, pen = H.gain_table(G, k, dev(part))
        b_o, p_o = orc.gain_table(h, k, part)
        assert np.array_equal(ben.cpu().numpy(), b_o)
        assert np.array_equal(pen.cpu().numpy(), p_o)


@pytest.mark.parametrize("name,k", CASES)
def test_gain_table_update_matches_oracle(hgp, orc, name, k):
    H = hgp
    h = make(name)
    G = H.Hypergraph.from_host(h)
    rs = np.random.RandomState(100 + k)
    for kind, part in partitions(orc, h, k, rs):
        for count in (1, 37, h.n // 3):
            say(f"[gains] update {name} k={k} {kind} moves={count}")
            us, ts = moves_of(rs, h, k, part, count, noop=min(3, count // 4))
            b0, p0 = orc.gain_table(h, k, part)
            part_o, b_o, p_o = orc.gain_table_moves(h, k, part, us, ts, b0, p0)
            t = dev(part)
            ben, pen = H.gain_table(G, k, t)
            H.gain_table_update(G, k, t, dev(us), dev(ts), ben, pen)
            assert np.array_equal(t.cpu().numpy().view(np.uint32), part_o)
            assert np.array_equal(ben.cpu().numpy(), b_o)
            assert np.array_equal(pen.cpu().numpy(), p_o)


@pytest.mark.parametrize("name,k", CASES)
def test_sequence_gains_match_oracle(hgp, orc, name, k):
    H = hgp
    h = make(name)
    G = H.Hypergraph.from_host(h)
    rs = np.random.RandomState(200 + k)
    for kind, part in partitions(orc, h, k, rs):
        for count in (1, 50, h.n // 2):
            say(f"[gains] recalc {name} k={k} {kind} moves={count}")
            us, ts = moves_of(rs, h, k, part, count, noop=min(2, count // 5))
            g_o = orc.gain_recalc(h, k, part, us, ts)
            t = dev(part)
            g = H.gain_recalc(G, k, t, dev(us), dev(ts))
            assert np.array_equal(g.cpu().numpy(), g_o)
            assert np.array_equal(t.cpu().numpy().view(np.uint32), part)  # left unchanged


def test_invalid_moves_rejected(hgp, orc):
    H = hgp
    h = make("random3k")
    k = 4
    G = H.Hypergraph.from_host(h)
    part = orc.greedy_ip(h, k)
    t = dev(part)
    ben, pen = H.gain_table(G, k, t)
    for us, ts in (([5, 9, 5], [1, 2, 3]), ([5, h.n], [1, 1]), ([5, 6], [1, k])):
        with pytest.raises(H.HGPError):
            H.gain_table_update(G, k, t, dev(us), dev(ts), ben, pen)
        with pytest.raises(H.HGPError):
            H.gain_recalc(G, k, t, dev(us), dev(ts))
    assert np.array_equal(t.cpu().numpy().view(np.uint32), part)
    b_o, p_o = orc.gain_table(h, k, part)
    assert np.array_equal(ben.cpu().numpy(), b_o) and np.array_equal(pen.cpu().numpy(), p_o)
