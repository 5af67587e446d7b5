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


def test_trusted_input_flag_gives_the_same_result(hgp, orc):
    h = W.random_uniform(4000, 4000, 2, 8, seed=12)
    G = hgp.Hypergraph.from_host(h)
    assert hgp.validate(G) == 0
    a = hgp.partition(G, hgp.params(4, seed=3))
    b = hgp.partition(G, hgp.params(4, seed=3, trusted=True))
    part_o, f_o, L_o = orc.partition(h, orc.params(4, seed=3))
    for part, f, L in (a, b):
        assert (f, L) == (f_o, L_o)
        assert np.array_equal(part.cpu().numpy().view(np.uint32), part_o)


def test_partition_workspace_too_small_for_the_hierarchy(hgp, orc):
    # a workspace smaller than one stored level: hgp_partition returns
    # HGP_E_WORKSPACE with its work drained, and the same output buffers then
    # give the oracle's result with a workspace of the documented size
    import torch
    H = hgp
    h = W.workload("stencil24")[0]
    k = 8
    G = H.Hypergraph.from_host(h)
    prm = H.params(k, seed=2)
    part_o, f_o, L_o = orc.partition(h, orc.params(k, seed=2))
    assert L_o >= 3
    level = 4 * (2 * G.m + 2 * G.p + 4 * G.n + 2)
    small = torch.empty(level // 2, dtype=torch.uint8, device="cuda")
    P = H.Partitioner(G, prm, ws=small)
    with pytest.raises(H.HGPError) as ei:
        P.run()
    assert ei.value.status == -3  # HGP_E_WORKSPACE
    P.ws = torch.empty(H.workspace_bytes(H.OP_PARTITION, G.n, G.m, G.p, prm), dtype=torch.uint8, device="cuda")
    L = P.run()
    assert (L, int(P.f.item())) == (L_o, f_o)
    assert np.array_equal(P.part.cpu().numpy().view(np.uint32), part_o)


@pytest.mark.parametrize("name,k,seed", [("stencil24", 8, 2), ("random120k", 2, 5), ("rmat16", 128, 4)])
def test_trace_matches_oracle_levels(hgp, orc, name, k, seed):
    # level sizes and LP rounds of hgp_partition_traced; random120k with
    # k = 2 hands a block pair of more than 4096 proposals to the
    # device-wide path in its last sub-rounds, which must not lose the count
    import test_gpu_parity as TP
    H = hgp
    h = TP.make(name)
    lv = orc.hierarchy(h, orc.params(k, seed=seed))
    G = H.Hypergraph.from_host(h)
    P = H.Partitioner(G, H.params(k, seed=seed))
    tr = P.run_traced()
    assert len(tr) == len(lv)
    for t, L in zip(tr, lv):
        assert (t["n"], t["m"], t["p"]) == (L["h"].n, L["h"].m, len(L["h"].pins))
        assert t["lp_rounds"] == L["lp_rounds"]


@pytest.mark.parametrize("rounds,subrounds", [(12, 5), (13, 5), (64, 1), (9, 8), (0, 5)])
def test_lp_candidate_list_paths(hgp, orc, rounds, subrounds):
    # Small levels list the candidates of every sub-round once per level when
    # rounds x sub-rounds <= 64 and select them per sub-round otherwise; both
    # must refine exactly as the oracle does, and so must whole partitions
    # (zero rounds: empty lists, nothing moves).
    h = W.random_uniform(3000, 3300, 2, 9, seed=17)
    k = 8
    part = W.uniform(W.rng(23, 0, np.arange(h.n, dtype=np.uint64)), k).astype(np.uint32)
    print(f"[rules] candidate lists rounds={rounds} subrounds={subrounds}", file=sys.stderr, flush=True)
    kw = dict(eps=(1, 10), seed=3, lp_rounds=rounds, lp_subrounds=subrounds)
    out_o, f_o, bw_o, rounds_o, moves_o = orc.refine_lp(h, orc.params(k, **kw), 0, part)
    G = hgp.Hypergraph.from_host(h)
    t = dev(part)
    f, bw = hgp.refine_lp(G, hgp.params(k, **kw), 0, t)
    assert f == f_o
    assert np.array_equal(t.cpu().numpy().view(np.uint32), out_o)
    assert bw.cpu().numpy().tolist() == bw_o.tolist()
    part_o, f_o, L_o = orc.partition(h, orc.params(k, **kw))
    p, f, L = hgp.partition(G, hgp.params(k, **kw))
    assert (L, f) == (L_o, f_o)
    assert np.array_equal(p.cpu().numpy().view(np.uint32), part_o)
