"""ctypes wrapper of the sequential CPU oracle (hgp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg; never by the partitioning library.
Hypergraphs are passed as any object with numpy attributes n, m, pin_off,
pins, inc_off, inc, vwgt, nwgt (uint32 IDs/offsets, int32 weights).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgp_oracle.c")
_LIB = os.path.join(_HERE, "libhgp_oracle.so")
NONE = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _HG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint32), ("p", ctypes.c_uint32),
                ("pin_off", ctypes.c_void_p), ("pins", ctypes.c_void_p),
                ("inc_off", ctypes.c_void_p), ("inc", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("nwgt", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("eps_num", ctypes.c_uint32), ("eps_den", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("limit_factor", ctypes.c_uint32),
                ("coarsen_subrounds", ctypes.c_uint32), ("lp_subrounds", ctypes.c_uint32),
                ("lp_rounds", ctypes.c_uint32), ("community", ctypes.c_uint32), ("ip", ctypes.c_uint32)]


def params(k: int, eps=(3, 100), seed: int = 0, limit_factor: int = 160,
           coarsen_subrounds: int = 3, lp_subrounds: int = 5, lp_rounds: int = 5, community: bool = False,
           ip: int = 0) -> Params:
    """ip: 0 greedy BFS fill, 1 recursive bipartitioning (Sec. 5)."""
    return Params(k, eps[0], eps[1], seed, limit_factor, coarsen_subrounds, lp_subrounds, lp_rounds,
                  1 if community else 0, ip)


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        u32, u64, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
        L.or_mix64.restype = u64; L.or_mix64.argtypes = [u64]
        L.or_hash.restype = u64; L.or_hash.argtypes = [u64, u32, u32, u32, u32]
        L.or_lmax.restype = i64; L.or_lmax.argtypes = [i64, u32, u32, u32]
        L.or_objective.restype = i64; L.or_objective.argtypes = [P, u32, P, P]
        L.or_gain.restype = i64; L.or_gain.argtypes = [P, P, u32, u32]
        L.or_rate_subround.restype = u32
        L.or_rate_subround.argtypes = [P, P, u32, u32, P, P, P, P]
        L.or_approve_apply.restype = u32; L.or_approve_apply.argtypes = [P, P, P, P, P, P]
        L.or_cluster_pass.restype = ctypes.c_int; L.or_cluster_pass.argtypes = [P, P, u32, P, P, P]
        L.or_contract.restype = ctypes.c_int
        L.or_contract.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.or_project.restype = None; L.or_project.argtypes = [u32, P, P, P]
        L.or_greedy_ip.restype = ctypes.c_int; L.or_greedy_ip.argtypes = [P, u32, P]
        L.or_select_pair.restype = ctypes.c_int
        L.or_select_pair.argtypes = [P, u32, P, u32, i64, i64, P, P]
        L.or_refine_lp.restype = ctypes.c_int
        L.or_refine_lp.argtypes = [P, P, u32, P, P, P, P, P]
        L.or_partition.restype = ctypes.c_int; L.or_partition.argtypes = [P, P, P, P, P]
        L.or_lp_proposals.restype = u32; L.or_lp_proposals.argtypes = [P, P, u32, u32, u32, P, P, P]
        L.or_gain_table.restype = ctypes.c_int; L.or_gain_table.argtypes = [P, u32, P, P, P]
        L.or_gain_table_moves.restype = ctypes.c_int
        L.or_gain_table_moves.argtypes = [P, u32, P, P, P, u32, P, P]
        L.or_gain_recalc.restype = ctypes.c_int; L.or_gain_recalc.argtypes = [P, u32, P, P, P, u32, P]
        L.or_graph_adjacency.restype = ctypes.c_int; L.or_graph_adjacency.argtypes = [P, P, P]
        L.or_graph_gain.restype = i64; L.or_graph_gain.argtypes = [P, P, P, P, u32, u32]
        L.or_graph_cut.restype = i64; L.or_graph_cut.argtypes = [P, P]
        L.or_graph_gain_table.restype = ctypes.c_int; L.or_graph_gain_table.argtypes = [P, u32, P, P]
        L.or_refine_lp_limits.restype = ctypes.c_int
        L.or_refine_lp_limits.argtypes = [P, P, u32, P, P, P, P, P, P]
        L.or_greedy_ip_targets.restype = ctypes.c_int; L.or_greedy_ip_targets.argtypes = [P, u32, P, P]
        L.or_lp_proposals_limits.restype = u32
        L.or_lp_proposals_limits.argtypes = [P, P, u32, u32, u32, P, P, P, P]
        L.or_rb_limits.restype = None; L.or_rb_limits.argtypes = [i64, u32, u32, u32, i64, u32, P, P]
        L.or_subhypergraph.restype = ctypes.c_int
        L.or_subhypergraph.argtypes = [P, P, u32, P, P, P, P, P, P, P, P]
        L.or_bisect.restype = ctypes.c_int; L.or_bisect.argtypes = [P, P, P, P, P]
        L.or_rb_ip.restype = ctypes.c_int; L.or_rb_ip.argtypes = [P, P, P]
        L.or_rate_subround_c.restype = u32
        L.or_rate_subround_c.argtypes = [P, P, u32, u32, P, P, P, P, P]
        L.or_cluster_pass_c.restype = ctypes.c_int; L.or_cluster_pass_c.argtypes = [P, P, u32, P, P, P, P]
        L.or_bipartite.restype = ctypes.c_int; L.or_bipartite.argtypes = [P, P, P, P, P, P, P]
        L.or_louvain_subround.restype = u32; L.or_louvain_subround.argtypes = [P, u64, u32, u32, u32, P, P]
        L.or_louvain_level.restype = u32; L.or_louvain_level.argtypes = [P, u64, u32, P, P]
        L.or_communities.restype = ctypes.c_int; L.or_communities.argtypes = [P, u64, P, P]
        L.or_graph_moves.restype = ctypes.c_int; L.or_graph_moves.argtypes = [P, u32, P, P, P, u32, P, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _View:
    """Keeps contiguous copies alive while the struct is in use."""

    def __init__(self, h):
        self.arrs = [np.ascontiguousarray(h.pin_off, np.uint32), np.ascontiguousarray(h.pins, np.uint32),
                     np.ascontiguousarray(h.inc_off, np.uint32), np.ascontiguousarray(h.inc, np.uint32),
                     np.ascontiguousarray(h.vwgt, np.int32), np.ascontiguousarray(h.nwgt, np.int32)]
        a = self.arrs
        self.s = _HG(int(h.n), int(h.m), int(a[1].shape[0]), *[a[i].ctypes.data for i in range(6)])

    @property
    def ref(self):
        return ctypes.byref(self.s)


def mix64(z: int) -> int:
    return lib().or_mix64(z)


def hash_(seed: int, purpose: int, level: int, it: int, x: int) -> int:
    return lib().or_hash(seed, purpose, level, it, x)


def lmax(W: int, k: int, eps=(3, 100)) -> int:
    return lib().or_lmax(W, k, eps[0], eps[1])


def objective(h, k: int, part: np.ndarray):
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    bw = np.zeros(k, np.int64)
    f = lib().or_objective(v.ref, k, _ptr(part), _ptr(bw))
    return int(f), bw


def gain(h, part: np.ndarray, u: int, t: int) -> int:
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    return int(lib().or_gain(v.ref, _ptr(part), u, t))


def rate_subround(h, P: Params, level: int, r: int, rep, cw, csize):
    v = _View(h)
    rep = np.ascontiguousarray(rep, np.uint32)
    cw = np.ascontiguousarray(cw, np.int64)
    csize = np.ascontiguousarray(csize, np.uint32)
    target = np.empty(h.n, np.uint32)
    nc = lib().or_rate_subround(v.ref, ctypes.byref(P), level, r, _ptr(rep), _ptr(cw), _ptr(csize), _ptr(target))
    return target, int(nc)


def rate_subround_c(h, P: Params, level: int, r: int, rep, cw, csize, comm):
    """rate_subround restricted to the communities comm (Sec. 4.3)."""
    v = _View(h)
    rep = np.ascontiguousarray(rep, np.uint32)
    cw = np.ascontiguousarray(cw, np.int64)
    csize = np.ascontiguousarray(csize, np.uint32)
    comm = np.ascontiguousarray(comm, np.uint32)
    target = np.empty(h.n, np.uint32)
    nc = lib().or_rate_subround_c(v.ref, ctypes.byref(P), level, r, _ptr(rep), _ptr(cw), _ptr(csize), _ptr(comm),
                                  _ptr(target))
    return target, int(nc)


def approve_apply(h, P: Params, target, rep, cw, csize) -> int:
    """Applies in place on rep (uint32), cw (int64), csize (uint32) arrays."""
    v = _View(h)
    assert rep.dtype == np.uint32 and cw.dtype == np.int64 and csize.dtype == np.uint32
    target = np.ascontiguousarray(target, np.uint32)
    return int(lib().or_approve_apply(v.ref, ctypes.byref(P), _ptr(target), _ptr(rep), _ptr(cw), _ptr(csize)))


def cluster_pass(h, P: Params, level: int):
    v = _View(h)
    rep = np.empty(h.n, np.uint32)
    cnt = np.zeros(1, np.uint32)
    run = np.zeros(1, np.uint32)
    rc = lib().or_cluster_pass(v.ref, ctypes.byref(P), level, _ptr(rep), _ptr(cnt), _ptr(run))
    assert rc == 0
    return rep, int(cnt[0]), int(run[0])


def cluster_pass_c(h, P: Params, level: int, comm):
    v = _View(h)
    comm = np.ascontiguousarray(comm, np.uint32)
    rep = np.empty(h.n, np.uint32)
    cnt = np.zeros(1, np.uint32)
    run = np.zeros(1, np.uint32)
    rc = lib().or_cluster_pass_c(v.ref, ctypes.byref(P), level, _ptr(comm), _ptr(rep), _ptr(cnt), _ptr(run))
    assert rc == 0
    return rep, int(cnt[0]), int(run[0])


def bipartite(h):
    """The bipartite graph G_x of h as a two-pin hypergraph namespace (node
    u < n: vertex u, node n + e: net e; vwgt = volumes), or None when its
    total volume reaches 2^31."""
    from types import SimpleNamespace
    v = _View(h)
    n, m, p = int(h.n), int(h.m), int(v.s.p)
    po = np.zeros(p + 1, np.uint32); pi = np.zeros(max(2 * p, 1), np.uint32)
    io = np.zeros(n + m + 1, np.uint32); ii = np.zeros(max(2 * p, 1), np.uint32)
    vw = np.zeros(max(n + m, 1), np.int32); nw = np.zeros(max(p, 1), np.int32)
    if lib().or_bipartite(v.ref, _ptr(po), _ptr(pi), _ptr(io), _ptr(ii), _ptr(vw), _ptr(nw)) != 0:
        return None
    return SimpleNamespace(n=n + m, m=p, pin_off=po, pins=pi[:2 * p], inc_off=io, inc=ii[:2 * p],
                           vwgt=vw[:n + m], nwgt=nw[:p])


def louvain_subround(g, seed: int, level: int, r: int, s: int, comm, cvol):
    """One synchronous local-moving sub-round; returns (moves, comm, cvol)."""
    v = _View(g)
    comm = np.array(comm, np.uint32)
    cvol = np.array(cvol, np.int64)
    mv = lib().or_louvain_subround(v.ref, seed, level, r, s, _ptr(comm), _ptr(cvol))
    return int(mv), comm, cvol


def louvain_level(g, seed: int, level: int):
    """Local moving of one level from singletons: (comm, moves, rounds)."""
    v = _View(g)
    comm = np.empty(max(g.n, 1), np.uint32)
    rounds = np.zeros(1, np.uint32)
    mv = lib().or_louvain_level(v.ref, seed, level, _ptr(comm), _ptr(rounds))
    return comm[:g.n], int(mv), int(rounds[0])


def communities(h, seed: int = 0):
    """Community of every vertex (Sec. 4.3) and the number of Louvain levels."""
    v = _View(h)
    comm = np.empty(max(h.n, 1), np.uint32)
    lv = np.zeros(1, np.uint32)
    rc = lib().or_communities(v.ref, seed, _ptr(comm), _ptr(lv))
    if rc != 0:
        raise ValueError("total volume of the bipartite graph reaches 2^31")
    return comm[:h.n], int(lv[0])


def contract(h, rep):
    """Returns (cid, coarse hypergraph as a HostHypergraph-like namespace)."""
    from types import SimpleNamespace
    v = _View(h)
    n, m, p = int(h.n), int(h.m), int(v.s.p)
    rep = np.ascontiguousarray(rep, np.uint32)
    cid = np.empty(n, np.uint32)
    dims = np.zeros(3, np.uint32)
    po = np.zeros(m + 1, np.uint32); pi = np.zeros(max(p, 1), np.uint32)
    io = np.zeros(n + 1, np.uint32); ii = np.zeros(max(p, 1), np.uint32)
    vw = np.zeros(max(n, 1), np.int32); nw = np.zeros(max(m, 1), np.int32)
    rc = lib().or_contract(v.ref, _ptr(rep), _ptr(cid), _ptr(dims), _ptr(po), _ptr(pi), _ptr(io), _ptr(ii),
                           _ptr(vw), _ptr(nw))
    assert rc == 0
    nc, mc, pc = (int(x) for x in dims)
    H = SimpleNamespace(n=nc, m=mc, pin_off=po[:mc + 1].copy(), pins=pi[:pc].copy(),
                        inc_off=io[:nc + 1].copy(), inc=ii[:pc].copy(), vwgt=vw[:nc].copy(),
                        nwgt=nw[:mc].copy())
    return cid, H


def project(cid, coarse_part):
    cid = np.ascontiguousarray(cid, np.uint32)
    cp = np.ascontiguousarray(coarse_part, np.uint32)
    out = np.empty(cid.shape[0], np.uint32)
    lib().or_project(cid.shape[0], _ptr(cid), _ptr(cp), _ptr(out))
    return out


def greedy_ip(h, k: int):
    v = _View(h)
    part = np.empty(h.n, np.uint32)
    assert lib().or_greedy_ip(v.ref, k, _ptr(part)) == 0
    return part


def select_pair(ca, cb, beta_s: int, beta_t: int):
    ca = np.ascontiguousarray(ca, np.int32)
    cb = np.ascontiguousarray(cb, np.int32)
    i = np.zeros(1, np.uint32); j = np.zeros(1, np.uint32)
    found = lib().or_select_pair(_ptr(ca), ca.shape[0], _ptr(cb), cb.shape[0], beta_s, beta_t, _ptr(i), _ptr(j))
    return bool(found), int(i[0]), int(j[0])


def refine_lp(h, P: Params, level: int, part):
    v = _View(h)
    part = np.array(part, dtype=np.uint32, copy=True)
    f = np.zeros(1, np.int64); bw = np.zeros(P.k, np.int64)
    rounds = np.zeros(1, np.uint32); moves = np.zeros(1, np.uint64)
    assert lib().or_refine_lp(v.ref, ctypes.byref(P), level, _ptr(part), _ptr(f), _ptr(bw), _ptr(rounds), _ptr(moves)) == 0
    return part, int(f[0]), bw, int(rounds[0]), int(moves[0])


def lp_proposals(h, P: Params, level: int, r: int, s: int, part):
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    t = np.empty(h.n, np.uint32)
    g = np.empty(h.n, np.int64)
    lib().or_lp_proposals(v.ref, ctypes.byref(P), level, r, s, _ptr(part), _ptr(t), _ptr(g))
    return t, g


def gain_table(h, k: int, part):
    """(benefit[n], penalty[n, k]) of the gain table (int64)."""
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    ben = np.zeros(max(h.n, 1), np.int64)
    pen = np.zeros((max(h.n, 1), k), np.int64)
    assert lib().or_gain_table(v.ref, k, _ptr(part), _ptr(ben), _ptr(pen)) == 0
    return ben[:h.n], pen[:h.n]


def gain_table_moves(h, k: int, part, mu, mt, ben, pen):
    """Applies the moves with the gain-table update rules; returns the new
    (part, benefit, penalty)."""
    v = _View(h)
    part = np.array(part, dtype=np.uint32, copy=True)
    ben = np.array(ben, dtype=np.int64, copy=True)
    pen = np.ascontiguousarray(np.array(pen, dtype=np.int64, copy=True))
    mu = np.ascontiguousarray(mu, np.uint32)
    mt = np.ascontiguousarray(mt, np.uint32)
    assert lib().or_gain_table_moves(v.ref, k, _ptr(part), _ptr(mu), _ptr(mt), mu.shape[0], _ptr(ben),
                                     _ptr(pen)) == 0
    return part, ben, pen


def gain_recalc(h, k: int, part, mu, mt):
    """Gain of every move of the sequence when performed in order (int64)."""
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    mu = np.ascontiguousarray(mu, np.uint32)
    mt = np.ascontiguousarray(mt, np.uint32)
    g = np.zeros(max(mu.shape[0], 1), np.int64)
    assert lib().or_gain_recalc(v.ref, k, _ptr(part), _ptr(mu), _ptr(mt), mu.shape[0], _ptr(g)) == 0
    return g[:mu.shape[0]]


def graph_adjacency(h):
    """(adj, adjw) of a hypergraph whose nets all have two pins, or None."""
    v = _View(h)
    p = int(v.s.p)
    adj = np.zeros(max(p, 1), np.uint32)
    adjw = np.zeros(max(p, 1), np.int32)
    if lib().or_graph_adjacency(v.ref, _ptr(adj), _ptr(adjw)) != 0:
        return None
    return adj[:p], adjw[:p]


def graph_gain(h, adj, adjw, part, u: int, t: int) -> int:
    v = _View(h)
    adj = np.ascontiguousarray(adj, np.uint32)
    adjw = np.ascontiguousarray(adjw, np.int32)
    part = np.ascontiguousarray(part, np.uint32)
    return int(lib().or_graph_gain(v.ref, _ptr(adj), _ptr(adjw), _ptr(part), u, t))


def graph_cut(h, part) -> int:
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    return int(lib().or_graph_cut(v.ref, _ptr(part)))


def graph_gain_table(h, k: int, part):
    """w(u, V_i) as an (n, k) int64 array, or None when a net has other than two pins."""
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    om = np.zeros((max(h.n, 1), k), np.int64)
    if lib().or_graph_gain_table(v.ref, k, _ptr(part), _ptr(om)) != 0:
        return None
    return om[:h.n]


def graph_moves(h, k: int, part, node, target, omega=None):
    """Moves made in order on a graph: returns (new part, attributed gains,
    updated omega or None).  Raises ValueError on invalid moves."""
    v = _View(h)
    part = np.array(part, np.uint32)
    node = np.ascontiguousarray(node, np.uint32)
    target = np.ascontiguousarray(target, np.uint32)
    g = np.zeros(max(len(node), 1), np.int64)
    om = None if omega is None else np.array(omega, np.int64).reshape(h.n, k)
    rc = lib().or_graph_moves(v.ref, k, _ptr(part), _ptr(node), _ptr(target), len(node),
                              None if om is None else _ptr(om), _ptr(g))
    if rc != 0:
        raise ValueError("invalid moves or not a graph")
    return part, g[:len(node)], om


def partition(h, P: Params):
    v = _View(h)
    part = np.empty(h.n, np.uint32)
    f = np.zeros(1, np.int64); lv = np.zeros(1, np.uint32)
    assert lib().or_partition(v.ref, ctypes.byref(P), _ptr(part), _ptr(f), _ptr(lv)) == 0
    return part, int(f[0]), int(lv[0])


def refine_lp_limits(h, P: Params, level: int, part, lmax):
    """LP with per-block weight limits: (part, f, bw, rounds, moves)."""
    v = _View(h)
    part = np.array(part, dtype=np.uint32, copy=True)
    lmax = np.ascontiguousarray(lmax, np.int64)
    f = np.zeros(1, np.int64); bw = np.zeros(P.k, np.int64)
    rounds = np.zeros(1, np.uint32); moves = np.zeros(1, np.uint64)
    assert lib().or_refine_lp_limits(v.ref, ctypes.byref(P), level, _ptr(part), _ptr(lmax), _ptr(f), _ptr(bw),
                                     _ptr(rounds), _ptr(moves)) == 0
    return part, int(f[0]), bw, int(rounds[0]), int(moves[0])


def lp_proposals_limits(h, P: Params, level: int, r: int, s: int, part, lmax):
    v = _View(h)
    part = np.ascontiguousarray(part, np.uint32)
    lmax = np.ascontiguousarray(lmax, np.int64)
    t = np.empty(h.n, np.uint32)
    g = np.empty(h.n, np.int64)
    lib().or_lp_proposals_limits(v.ref, ctypes.byref(P), level, r, s, _ptr(part), _ptr(lmax), _ptr(t), _ptr(g))
    return t, g


def greedy_ip_targets(h, k: int, targets):
    v = _View(h)
    t = np.ascontiguousarray(targets, np.int64)
    part = np.empty(max(h.n, 1), np.uint32)
    assert lib().or_greedy_ip_targets(v.ref, k, _ptr(t), _ptr(part)) == 0
    return part[:h.n]


def rb_limits(Wtot: int, ktot: int, eps, Wsub: int, kk: int):
    """(L[2], T[2]) of a bisection (Eq. 1)."""
    L = np.zeros(2, np.int64); T = np.zeros(2, np.int64)
    lib().or_rb_limits(Wtot, ktot, eps[0], eps[1], Wsub, kk, _ptr(L), _ptr(T))
    return L.tolist(), T.tolist()


def subhypergraph(h, part, side: int):
    """(H[V_side] as a namespace, vmap)."""
    from types import SimpleNamespace
    v = _View(h)
    n, m, p = int(h.n), int(h.m), int(v.s.p)
    part = np.ascontiguousarray(part, np.uint32)
    dims = np.zeros(3, np.uint32)
    po = np.zeros(m + 1, np.uint32); pi = np.zeros(max(p, 1), np.uint32)
    io = np.zeros(n + 1, np.uint32); ii = np.zeros(max(p, 1), np.uint32)
    vw = np.zeros(max(n, 1), np.int32); nw = np.zeros(max(m, 1), np.int32)
    vm = np.zeros(max(n, 1), np.uint32)
    assert lib().or_subhypergraph(v.ref, _ptr(part), side, _ptr(dims), _ptr(po), _ptr(pi), _ptr(io), _ptr(ii),
                                  _ptr(vw), _ptr(nw), _ptr(vm)) == 0
    n2, m2, p2 = (int(x) for x in dims)
    H = SimpleNamespace(n=n2, m=m2, pin_off=po[:m2 + 1].copy(), pins=pi[:p2].copy(), inc_off=io[:n2 + 1].copy(),
                        inc=ii[:p2].copy(), vwgt=vw[:n2].copy(), nwgt=nw[:m2].copy())
    return H, vm[:n2].copy()


def bisect(h, P: Params, L, T):
    v = _View(h)
    L = np.ascontiguousarray(L, np.int64); T = np.ascontiguousarray(T, np.int64)
    part = np.empty(max(h.n, 1), np.uint32)
    assert lib().or_bisect(v.ref, ctypes.byref(P), _ptr(L), _ptr(T), _ptr(part)) == 0
    return part[:h.n]


def rb_ip(h, P: Params):
    """Recursive-bipartitioning initial partition (Sec. 5) of h into P.k blocks."""
    v = _View(h)
    part = np.empty(max(h.n, 1), np.uint32)
    assert lib().or_rb_ip(v.ref, ctypes.byref(P), _ptr(part)) == 0
    return part[:h.n]


def hierarchy(h, P: Params):
    """The oracle's multilevel driver taken level by level (same steps as
    or_partition), returning every intermediate array for per-level parity:
    list of dicts with the level hypergraph, rep, cnt, cid, and the refined
    partition of every level."""
    levels = [{"h": h}]
    cur = h
    comm = communities(h, P.seed)[0] if P.community else None
    while cur.n > P.limit_factor * P.k:
        lvl = len(levels) - 1
        if comm is not None:
            levels[-1]["comm"] = comm
            rep, cnt, run = cluster_pass_c(cur, P, lvl, comm)
        else:
            rep, cnt, run = cluster_pass(cur, P, lvl)
        levels[-1].update(rep=rep, cnt=cnt, subrounds=run)
        if 100 * (cur.n - cnt) <= cur.n:
            break
        cid, H = contract(cur, rep)
        levels[-1]["cid"] = cid
        levels.append({"h": H})
        if comm is not None:
            nxt = np.zeros(H.n, np.uint32)
            nxt[cid] = comm
            comm = nxt
        cur = H
    L = len(levels) - 1
    part = rb_ip(cur, P) if P.ip == 1 else greedy_ip(cur, P.k)
    levels[L]["ip"] = part.copy()
    part, f, bw, rounds, moves = refine_lp(cur, P, L, part)
    levels[L].update(part=part, f=f, bw=bw, lp_rounds=rounds, lp_moves=moves)
    for l in range(L - 1, -1, -1):
        proj = project(levels[l]["cid"], part)
        levels[l]["proj"] = proj
        part, f, bw, rounds, moves = refine_lp(levels[l]["h"], P, l, proj)
        levels[l].update(part=part, f=f, bw=bw, lp_rounds=rounds, lp_moves=moves)
    return levels
