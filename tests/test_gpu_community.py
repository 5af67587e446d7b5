"""GPU parity of the community detection (Sec. 4.3, deterministic Louvain of
Sec. 11) and of community-aware partitioning against the oracle, through the
C ABI: the community of every vertex, the number of Louvain levels, and the
final partition, objective and level sizes of hgp_partition with
params.community = 1."""
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


def make(name):
    rs = np.random.RandomState(23)
    if name == "random2k":
        return W.random_uniform(2000, 2000, 2, 8, seed=9, name=name)
    if name == "hugenets":  # sorted runs of more than 64 entries: the wave paths
        n = 4000
        nets = [rs.choice(n, size=rs.randint(2, 7), replace=False) for _ in range(4000)]
        nets += [rs.choice(n, size=sz, replace=False) for sz in (40, 90, 300, 1500)]
        return W.from_nets(n, nets, nwgt=rs.randint(1, 4, size=len(nets)))
    if name == "singles":  # single-pin nets and isolated vertices
        nets = [[v] for v in range(0, 300, 7)] + [sorted(rs.choice(300, 3, replace=False).tolist())
                                                   for _ in range(250)]
        return W.from_nets(330, nets)
    return W.workload(name)[0]


CASES = ["random2k", "stencil16", "powerlaw20000", "hugenets", "singles", "rmat16", "stencil32"]


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("seed", [0, 7])
def test_communities_match_oracle(hgp, orc, name, seed):
    H = hgp
    h = make(name)
    say(f"[communities] {name} seed={seed} n={h.n} m={h.m}")
    comm_o, lv_o = orc.communities(h, seed)
    comm, lv = H.communities(H.Hypergraph.from_host(h), seed)
    assert lv == lv_o
    assert np.array_equal(comm.cpu().numpy().view(np.uint32), comm_o)


PART_CASES = [("random2k", 2, 1), ("stencil16", 8, 2), ("powerlaw20000", 8, 3), ("hugenets", 4, 4),
              ("stencil32", 64, 5)]


@pytest.mark.parametrize("name,k,seed", PART_CASES)
def test_community_partition_matches_oracle(hgp, orc, name, k, seed):
    H = hgp
    h = make(name)
    P_or = orc.params(k, seed=seed, community=True)
    lv = orc.hierarchy(h, P_or)
    part_o, f_o, L_o = orc.partition(h, P_or)
    say(f"[community partition] {name} k={k} levels={L_o}")
    G = H.Hypergraph.from_host(h)
    P = H.Partitioner(G, H.params(k, seed=seed, community=True))
    tr = P.run_traced()
    assert [(t["n"], t["m"], t["p"]) for t in tr] == [(L["h"].n, L["h"].m, len(L["h"].pins)) for L in lv]
    assert int(P.f.item()) == f_o and len(tr) - 1 == L_o
    assert np.array_equal(P.part.cpu().numpy().view(np.uint32), part_o)


def test_volume_bound_rejected(hgp):
    H = hgp
    h = W.from_nets(3, [[0, 1, 2], [0, 1]], nwgt=[1 << 29, 1])  # total volume 2 (3 2^29 + 2) >= 2^31
    with pytest.raises(H.HGPError):
        H.communities(H.Hypergraph.from_host(h))
    with pytest.raises(H.HGPError):
        H.partition(H.Hypergraph.from_host(h), H.params(2, community=True))
