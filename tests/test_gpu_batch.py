"""Many hypergraphs at once: hgp_partition_batch and the partition server.

Every request must give exactly what hgp_partition gives on its own (and what
the oracle gives), whatever else runs beside it: the batch is checked against
the oracle instance by instance, and the server against single calls while
requests of mixed sizes compete for lanes and pool memory.
"""
import sys

import numpy as np
import pytest

from paper_2303_17679_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hgp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_17679_amd as H
    H.lib()
    return H


def host(t):
    return t.cpu().numpy().view(np.uint32)


def small_vlsi(count, nmax=30000):
    """The first `count` batch-workload instances with n <= nmax."""
    ns, ks = W.vlsi_params(512)
    out = []
    for i in range(512):
        if ns[i] <= nmax:
            out.append((W.vlsi(int(ns[i]), i), int(ks[i]), i))
        if len(out) == count:
            break
    return out


def test_batch_matches_oracle(hgp, orc):
    H = hgp
    inst = small_vlsi(12)
    hs = [H.Hypergraph.from_host(h) for h, _, _ in inst]
    prms = [H.params(k, seed=i) for (_, k, i) in inst]
    say(f"[batch] {len(inst)} instances, n = {[h.n for h, _, _ in inst]}")
    parts, objs, levels = H.partition_batch(hs, prms, lanes=4)
    objs = objs.cpu().numpy()
    for j, (h, k, i) in enumerate(inst):
        part_o, f_o, L_o = orc.partition(h, orc.params(k, seed=i))
        assert (int(objs[j]), levels[j]) == (f_o, L_o), j
        assert np.array_equal(host(parts[j]), part_o), j


def test_batch_one_lane_and_tight_workspace(hgp):
    H = hgp
    inst = small_vlsi(5)
    hs = [H.Hypergraph.from_host(h) for h, _, _ in inst]
    prms = [H.params(k, seed=1) for (_, k, _) in inst]
    ref = [H.partition(g, p) for g, p in zip(hs, prms)]
    # the smallest workspace the batch accepts: one request at a time
    import ctypes
    HG = H._HG * len(hs)
    PA = H.Params * len(hs)
    need = ctypes.c_size_t(0)
    assert H.lib().hgp_batch_workspace_bytes(HG(*[g.struct() for g in hs]), PA(*prms), len(hs), 1,
                                             ctypes.byref(need)) == 0
    parts, objs, levels = H.partition_batch(hs, prms, lanes=3, ws_bytes=int(need.value))
    for j, (p_ref, f_ref, l_ref) in enumerate(ref):
        assert np.array_equal(host(parts[j]), host(p_ref)) and int(objs[j]) == f_ref and levels[j] == l_ref


def test_server_same_alone_and_in_the_mix(hgp):
    import torch
    H = hgp
    reqs = [(W.workload("stencil24")[0], 16, 1), (W.workload("powerlaw20000")[0], 8, 2),
            (W.random_uniform(5000, 5000, 2, 8, seed=5), 2, 3), (W.workload("stencil16")[0], 4, 4)]
    reqs += [(h, k, 10 + i) for (h, k, i) in small_vlsi(6)]
    hs = [H.Hypergraph.from_host(h) for h, _, _ in reqs]
    prms = [H.params(k, seed=sd) for (_, k, sd) in reqs]
    alone = [H.partition(g, p) for g, p in zip(hs, prms)]
    need = [H.workspace_bytes(H.OP_PARTITION, g.n, g.m, g.p, p) for g, p in zip(hs, prms)]
    # a pool that holds the two largest requests but not all of them: some
    # requests wait for memory, smaller ones may pass them
    pool = sorted(need)[-1] + sorted(need)[-2] + 4096
    say(f"[server] {len(reqs)} requests, pool {pool} bytes, needs {need}")
    S = H.Server(lanes=4, pool_bytes=pool)
    try:
        for rep in range(2):
            tickets = [S.submit(g, p) for g, p in zip(hs, prms)]
            for (t, part, obj), (p_ref, f_ref, l_ref) in zip(tickets, alone):
                lv, lat, qm = S.wait(t)
                torch.cuda.synchronize()
                assert lv == l_ref and int(obj.item()) == f_ref
                assert np.array_equal(host(part), host(p_ref))
                assert lat >= qm >= 0
    finally:
        S.close()


def test_server_rejects_request_larger_than_pool(hgp):
    H = hgp
    g = H.Hypergraph.from_host(W.workload("stencil16")[0])
    prm = H.params(4)
    S = H.Server(lanes=1, pool_bytes=1 << 16)
    try:
        with pytest.raises(H.HGPError):
            S.submit(g, prm)
    finally:
        S.close()


def test_server_failed_requests_leave_the_others_intact(hgp):
    # malformed requests (pins out of order, so the device-side validation
    # fails after launching its kernels) mixed with good ones: every failed
    # request returns its error after its own work has drained, the pool
    # memory it held goes to later requests, and every good request equals
    # its result alone
    import dataclasses
    import torch
    H = hgp
    good = [(W.workload("stencil16")[0], 4, 4), (W.random_uniform(5000, 5000, 2, 8, seed=5), 2, 3)]
    good += [(h, k, 10 + i) for (h, k, i) in small_vlsi(4)]
    bad_h = W.random_uniform(20000, 20000, 2, 8, seed=7)
    pins = bad_h.pins.copy()
    a, b = int(bad_h.pin_off[10]), int(bad_h.pin_off[10]) + 1
    pins[a], pins[b] = pins[b], pins[a]
    bad_h = dataclasses.replace(bad_h, pins=pins)
    hs = [H.Hypergraph.from_host(h) for h, _, _ in good]
    prms = [H.params(k, seed=sd) for (_, k, sd) in good]
    alone = [H.partition(g, p) for g, p in zip(hs, prms)]
    bad = H.Hypergraph.from_host(bad_h)
    with pytest.raises(H.HGPError):
        H.partition(bad, H.params(8))
    need = [H.workspace_bytes(H.OP_PARTITION, g.n, g.m, g.p, p) for g, p in zip(hs, prms)]
    need_bad = H.workspace_bytes(H.OP_PARTITION, bad.n, bad.m, bad.p, H.params(8))
    pool = max(need + [need_bad]) * 2 + 4096
    S = H.Server(lanes=3, pool_bytes=pool)
    try:
        order = []
        for i, (g, p) in enumerate(zip(hs, prms)):
            order.append(("bad", S.submit(bad, H.params(8))))
            order.append((i, S.submit(g, p)))
        for what, (t, part, obj) in order:
            if what == "bad":
                with pytest.raises(H.HGPError) as ei:
                    S.wait(t)
                assert ei.value.status == -1  # HGP_E_INVALID
                continue
            lv, lat, qm = S.wait(t)
            torch.cuda.synchronize()
            p_ref, f_ref, l_ref = alone[what]
            assert lv == l_ref and int(obj.item()) == f_ref
            assert np.array_equal(host(part), host(p_ref))
    finally:
        S.close()


def test_batch_many_small_instances(hgp, orc):
    # Many small instances on 16 lanes, with one to four Lambda words and
    # several sub-round and round counts. Every result equals the oracle's
    # and the one-at-a-time result.
    H = hgp
    rs = np.random.RandomState(77)
    inst = []
    for i in range(40):
        n = int(rs.randint(200, 4500))
        k = int(rs.choice([2, 3, 8, 64, 100, 200]))
        h = W.random_uniform(n, n + int(rs.randint(0, n // 2)), 2, 8, seed=100 + i, name=f"r{i}")
        kw = {"lp_subrounds": int(rs.choice([1, 5, 7])), "lp_rounds": int(rs.choice([1, 5, 9]))}
        if k >= 64:
            kw["eps"] = (1, 2)  # room to move with few vertices per block
        inst.append((h, k, i, kw))
    hs = [H.Hypergraph.from_host(h) for h, _, _, _ in inst]
    prms = [H.params(k, seed=i, **kw) for (_, k, i, kw) in inst]
    say(f"[batch small] {len(inst)} instances on 16 lanes")
    parts, objs, levels = H.partition_batch(hs, prms, lanes=16)
    for j, (h, k, i, kw) in enumerate(inst):
        part_o, f_o, L_o = orc.partition(h, orc.params(k, seed=i, **kw))
        assert (int(objs[j].item()), levels[j]) == (f_o, L_o), j
        assert np.array_equal(host(parts[j]), part_o), j
    for j in (0, 7, 19):
        part, f, L = H.partition(hs[j], prms[j])
        assert (f, L) == (int(objs[j].item()), levels[j]) and np.array_equal(host(part), host(parts[j]))
