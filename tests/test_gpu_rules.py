"""GPU parity on the control-rule fixtures of the oracle: the LP round without
moves, the swap that only one sub-round grouping allows, the 1 % contraction
stop and the pass cut at exactly n/2.5, through the C ABI."""
import sys

import numpy as np
import pytest

import bruteforce as bf
import test_oracle_rules as R
from paper_2303_17679_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_17679_amd as H
    H.lib()
    return H


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("together,rounds,moves", [([False, True], 1, 0), ([True], 2, 2)])
def test_lp_rounds_and_swap(hgp, orc, together, rounds, moves):
    h, part = R.swap_instance()
    seed = R._seed_for(together)
    print(f"[rules] swap instance seed={seed}", file=sys.stderr, flush=True)
    P_or = orc.params(3, eps=(1, 10), seed=seed, lp_rounds=5, lp_subrounds=2)
    out_o, f_o, bw_o, rounds_o, moves_o = orc.refine_lp(h, P_or, 0, part)
    assert (rounds_o, moves_o) == (rounds, moves)
    G = hgp.Hypergraph.from_host(h)
    t = dev(part)
    f, bw = hgp.refine_lp(G, hgp.params(3, eps=(1, 10), seed=seed, lp_rounds=5, lp_subrounds=2), 0, t)
    assert f == f_o
    assert np.array_equal(t.cpu().numpy().view(np.uint32), out_o)
    assert bw.cpu().numpy().tolist() == bw_o.tolist()


@pytest.mark.parametrize("n,joins,contracts", [(100, 1, False), (100, 2, True), (200, 2, False), (200, 3, True)])
def test_one_percent_rule(hgp, orc, n, joins, contracts):
    seed = 5
    h = W.from_nets(n, R._pairs_in_different_subrounds(seed, n, joins))
    print(f"[rules] one percent n={n} joins={joins}", file=sys.stderr, flush=True)
    part_o, f_o, L_o = orc.partition(h, orc.params(2, seed=seed, limit_factor=1))
    assert (L_o >= 1) == contracts
    G = hgp.Hypergraph.from_host(h)
    part, f, L = hgp.partition(G, hgp.params(2, seed=seed, limit_factor=1))
    assert (L, f) == (L_o, f_o)
    assert np.array_equal(part.cpu().numpy().view(np.uint32), part_o)


def test_pass_cut_boundary_cases(hgp, orc):
    # the replayed pass-cut cases: cluster counts and representatives equal
    # the oracle's for every case, including the equality boundary
    eq_h, eq_seed, eq_sc, _, _ = R.equality_case()
    cases = R._pass_cases() + [(eq_h, eq_sc, eq_seed)]
    for h, sc, seed in cases:
        P_or = orc.params(2, seed=seed, limit_factor=1, coarsen_subrounds=sc)
        rep_o, cnt_o, run_o = orc.cluster_pass(h, P_or, 0)
        G = hgp.Hypergraph.from_host(h)
        rep, cnt = hgp.coarsen(G, hgp.params(2, seed=seed, limit_factor=1, coarsen_subrounds=sc), 0)
        assert cnt == cnt_o
        assert np.array_equal(rep.cpu().numpy().view(np.uint32), rep_o)
