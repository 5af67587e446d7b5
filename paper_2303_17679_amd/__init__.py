"""Python binding of libhgp.so, the gfx950 multilevel hypergraph partitioning
hot path (coarsening, contraction, deterministic label propagation) of
"Scalable High-Quality Hypergraph Partitioning" (arXiv 2303.17679).

Argument marshalling only: every step runs in the HIP library.  PyTorch
provides device memory (int32 tensors holding uint32 IDs) and the current
stream.  If the library is not built, every call raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgp.so")

OP_COARSEN, OP_CONTRACT, OP_REFINE, OP_PARTITION, OP_VALIDATE, OP_INITIAL, OP_GAINS, OP_COMMUNITY, OP_RB = \
    1, 2, 3, 4, 5, 6, 7, 8, 9
STATUS = {0: "HGP_OK", -1: "HGP_E_INVALID", -2: "HGP_E_OVERFLOW", -3: "HGP_E_WORKSPACE",
          -4: "HGP_E_DEVICE", -5: "HGP_E_UNSUPPORTED"}

EXPORTS = ["hgp_default_params", "hgp_workspace_bytes", "hgp_validate", "hgp_coarsen", "hgp_contract",
           "hgp_project", "hgp_objective", "hgp_refine_lp", "hgp_initial_partition", "hgp_partition",
           "hgp_timing_scratch_bytes", "hgp_timing_begin", "hgp_timing_sample", "hgp_timing_end",
           "hgp_status_str",
           "hgp_server_create", "hgp_server_submit", "hgp_server_wait", "hgp_server_destroy",
           "hgp_batch_workspace_bytes", "hgp_partition_batch", "hgp_refine_lp_static",
           "hgp_partition_traced", "hgp_gain_table", "hgp_gain_table_update", "hgp_gain_recalc",
           "hgp_graph_gain_table", "hgp_graph_moves", "hgp_communities", "hgp_rb_initial_partition"]

# kernel ids of the measurement calls, with the kernel symbol each one names
KERNELS = ["k_rate_group<8, 64, 6>", "k_rate_group<16, 256, 8>", "k_rate_group<64, 1024, 10>", "k_rate_block",
           "k_gains", "k_lp_fast", "k_lp_pairs", "k_lp_update_movers", "k_hub_insert", "k_hub_argmax", "k_hub_lds"]


class HGPError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_status_str(status)})")


class _HG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint32), ("p", ctypes.c_uint32),
                ("pin_off", ctypes.c_void_p), ("pins", ctypes.c_void_p),
                ("inc_off", ctypes.c_void_p), ("inc", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("nwgt", ctypes.c_void_p)]


class _HGOut(ctypes.Structure):
    _fields_ = [("cap_n", ctypes.c_uint32), ("cap_m", ctypes.c_uint32), ("cap_p", ctypes.c_uint32),
                ("pin_off", ctypes.c_void_p), ("pins", ctypes.c_void_p),
                ("inc_off", ctypes.c_void_p), ("inc", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("nwgt", ctypes.c_void_p), ("dims", ctypes.c_void_p)]


class _Trace(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_uint32), ("levels", ctypes.c_uint32),
                ("n", ctypes.c_void_p), ("m", ctypes.c_void_p), ("p", ctypes.c_void_p),
                ("lp_rounds", ctypes.c_void_p)]


class Params(ctypes.Structure):
    """Mirror of hgp_params (every field changes results)."""
    _fields_ = [("k", ctypes.c_uint32), ("eps_num", ctypes.c_uint32), ("eps_den", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("limit_factor", ctypes.c_uint32),
                ("coarsen_subrounds", ctypes.c_uint32), ("lp_subrounds", ctypes.c_uint32),
                ("lp_rounds", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("community", ctypes.c_uint32),
                ("ip", ctypes.c_uint32)]


def params(k: int, eps=(3, 100), seed: int = 0, limit_factor: int = 160, coarsen_subrounds: int = 3,
           lp_subrounds: int = 5, lp_rounds: int = 5, trusted: bool = False, community: bool = False,
           ip: int = 0) -> Params:
    """trusted: the input was validated before (hgp_validate), so
    hgp_partition skips its own input check (HGP_TRUSTED_INPUT).
    community: community-aware coarsening (hgp_communities first).
    ip: initial partition of the coarsest level, 0 greedy BFS fill, 1
    recursive bipartitioning (Sec. 5, Eq. 1)."""
    return Params(k, eps[0], eps[1], seed, limit_factor, coarsen_subrounds, lp_subrounds, lp_rounds,
                  1 if trusted else 0, 1 if community else 0, ip)


_lib = None


def lib():
    """Load libhgp.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2303_17679_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32
        L.hgp_default_params.restype = i32; L.hgp_default_params.argtypes = [u32, P]
        L.hgp_workspace_bytes.restype = i32
        L.hgp_workspace_bytes.argtypes = [ctypes.c_int, u32, u32, u32, P, ctypes.POINTER(ctypes.c_size_t)]
        L.hgp_validate.restype = i32; L.hgp_validate.argtypes = [P, P, ctypes.c_size_t, P]
        L.hgp_coarsen.restype = i32; L.hgp_coarsen.argtypes = [P, P, u32, P, P, P, ctypes.c_size_t, P]
        L.hgp_contract.restype = i32; L.hgp_contract.argtypes = [P, P, P, P, P, ctypes.c_size_t, P]
        L.hgp_project.restype = i32; L.hgp_project.argtypes = [u32, P, P, P, P]
        L.hgp_objective.restype = i32; L.hgp_objective.argtypes = [P, u32, P, P, P, P, ctypes.c_size_t, P]
        L.hgp_refine_lp.restype = i32; L.hgp_refine_lp.argtypes = [P, P, u32, P, P, P, P, ctypes.c_size_t, P]
        L.hgp_refine_lp_static.restype = i32; L.hgp_refine_lp_static.argtypes = [P, P, u32, P, P, P, P]
        L.hgp_initial_partition.restype = i32
        L.hgp_initial_partition.argtypes = [P, u32, P, P, ctypes.c_size_t, P]
        L.hgp_rb_initial_partition.restype = i32
        L.hgp_rb_initial_partition.argtypes = [P, P, P, P, ctypes.c_size_t, P]
        L.hgp_partition.restype = i32
        L.hgp_partition.argtypes = [P, P, P, P, ctypes.POINTER(ctypes.c_uint32), P, ctypes.c_size_t, P]
        L.hgp_gain_table.restype = i32; L.hgp_gain_table.argtypes = [P, u32, P, P, P, P, ctypes.c_size_t, P]
        L.hgp_gain_table_update.restype = i32
        L.hgp_gain_table_update.argtypes = [P, u32, P, P, P, u32, P, P, P, ctypes.c_size_t, P]
        L.hgp_gain_recalc.restype = i32
        L.hgp_gain_recalc.argtypes = [P, u32, P, P, P, u32, P, P, ctypes.c_size_t, P]
        L.hgp_communities.restype = i32
        L.hgp_communities.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(ctypes.c_uint32), P, ctypes.c_size_t, P]
        L.hgp_graph_gain_table.restype = i32
        L.hgp_graph_gain_table.argtypes = [P, u32, P, P, P, ctypes.c_size_t, P]
        L.hgp_graph_moves.restype = i32
        L.hgp_graph_moves.argtypes = [P, u32, P, P, P, u32, P, P, P, ctypes.c_size_t, P]
        L.hgp_partition_traced.restype = i32
        L.hgp_partition_traced.argtypes = [P, P, P, P, P, P, ctypes.c_size_t, P]
        L.hgp_status_str.restype = ctypes.c_char_p; L.hgp_status_str.argtypes = [i32]
        L.hgp_timing_scratch_bytes.restype = i32
        L.hgp_timing_scratch_bytes.argtypes = [u32, u32, ctypes.POINTER(ctypes.c_size_t)]
        L.hgp_timing_begin.restype = i32
        L.hgp_timing_begin.argtypes = [u32, ctypes.c_int, P, ctypes.c_size_t, u32, u32]
        L.hgp_timing_sample.restype = i32; L.hgp_timing_sample.argtypes = [u32, u32]
        L.hgp_timing_end.restype = i32
        L.hgp_timing_end.argtypes = [u32, P, P, P]
        L.hgp_server_create.restype = i32
        L.hgp_server_create.argtypes = [u32, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
        L.hgp_server_submit.restype = i32
        L.hgp_server_submit.argtypes = [P, P, P, P, P, P, ctypes.POINTER(ctypes.c_uint64)]
        L.hgp_server_wait.restype = i32
        L.hgp_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.hgp_server_destroy.restype = i32; L.hgp_server_destroy.argtypes = [P]
        L.hgp_batch_workspace_bytes.restype = i32
        L.hgp_batch_workspace_bytes.argtypes = [P, P, u32, u32, ctypes.POINTER(ctypes.c_size_t)]
        L.hgp_partition_batch.restype = i32
        L.hgp_partition_batch.argtypes = [P, P, u32, u32, P, P, P, P, ctypes.c_size_t, P]
        _lib = L
    return _lib


def _status_str(s: int) -> str:
    try:
        return lib().hgp_status_str(s).decode()
    except Exception:  # library missing: still report the code
        return str(s)


def _check(s: int, what: str):
    if s != 0:
        raise HGPError(s, what)


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


@dataclass
class Hypergraph:
    """Device-resident level: int32 tensors (uint32 values) on a GPU."""
    n: int
    m: int
    p: int
    pin_off: object
    pins: object
    inc_off: object
    inc: object
    vwgt: object
    nwgt: object

    @classmethod
    def from_host(cls, h, device="cuda"):
        torch = _torch()

        def t(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(device)
        return cls(int(h.n), int(h.m), int(len(h.pins)), t(h.pin_off, np.int32), t(h.pins, np.int32),
                   t(h.inc_off, np.int32), t(h.inc, np.int32), t(h.vwgt, np.int32), t(h.nwgt, np.int32))

    def to_host(self):
        from types import SimpleNamespace

        def a(x):
            return x.cpu().numpy().view(np.uint32)
        return SimpleNamespace(n=self.n, m=self.m, pin_off=a(self.pin_off), pins=a(self.pins),
                               inc_off=a(self.inc_off), inc=a(self.inc),
                               vwgt=self.vwgt.cpu().numpy().astype(np.int32),
                               nwgt=self.nwgt.cpu().numpy().astype(np.int32))

    def struct(self) -> _HG:
        return _HG(self.n, self.m, self.p, _ptr(self.pin_off), _ptr(self.pins), _ptr(self.inc_off),
                   _ptr(self.inc), _ptr(self.vwgt), _ptr(self.nwgt))

    @property
    def device(self):
        return self.pin_off.device


def workspace_bytes(op: int, n: int, m: int, p: int, prm: Params | None = None) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().hgp_workspace_bytes(op, n, m, p, ctypes.byref(prm) if prm is not None else None,
                                     ctypes.byref(out)), "hgp_workspace_bytes")
    return int(out.value)


def _ws(op, h: Hypergraph, prm=None):
    torch = _torch()
    nb = workspace_bytes(op, h.n, h.m, h.p, prm)
    return torch.empty(nb, dtype=torch.uint8, device=h.device)


def validate(h: Hypergraph) -> int:
    ws = _ws(OP_VALIDATE, h)
    s = h.struct()
    return int(lib().hgp_validate(ctypes.byref(s), _ptr(ws), ws.numel(), _stream()))


def coarsen(h: Hypergraph, prm: Params, level: int = 0):
    """One clustering pass; returns (rep tensor, number of clusters)."""
    torch = _torch()
    rep = torch.empty(h.n, dtype=torch.int32, device=h.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=h.device)
    ws = _ws(OP_COARSEN, h, prm)
    s = h.struct()
    _check(lib().hgp_coarsen(ctypes.byref(s), ctypes.byref(prm), level, _ptr(rep), _ptr(cnt), _ptr(ws),
                             ws.numel(), _stream()), "hgp_coarsen")
    return rep, int(cnt.item())


def contract(h: Hypergraph, rep):
    """Contract a clustering; returns (cid tensor, coarse Hypergraph)."""
    torch = _torch()
    dev = h.device
    cid = torch.empty(h.n, dtype=torch.int32, device=dev)
    bufs = dict(pin_off=torch.empty(h.m + 1, dtype=torch.int32, device=dev),
                pins=torch.empty(max(h.p, 1), dtype=torch.int32, device=dev),
                inc_off=torch.empty(h.n + 1, dtype=torch.int32, device=dev),
                inc=torch.empty(max(h.p, 1), dtype=torch.int32, device=dev),
                vwgt=torch.empty(h.n, dtype=torch.int32, device=dev),
                nwgt=torch.empty(max(h.m, 1), dtype=torch.int32, device=dev))
    dims = torch.zeros(3, dtype=torch.int32, device=dev)
    out = _HGOut(h.n, h.m, h.p, *[_ptr(bufs[k]) for k in ("pin_off", "pins", "inc_off", "inc", "vwgt", "nwgt")],
                 _ptr(dims))
    ws = _ws(OP_CONTRACT, h)
    s = h.struct()
    _check(lib().hgp_contract(ctypes.byref(s), _ptr(rep), _ptr(cid), ctypes.byref(out), _ptr(ws), ws.numel(),
                              _stream()), "hgp_contract")
    nc, mc, pc = (int(x) for x in dims.cpu().tolist())
    H = Hypergraph(nc, mc, pc, bufs["pin_off"][:mc + 1], bufs["pins"][:pc], bufs["inc_off"][:nc + 1],
                   bufs["inc"][:pc], bufs["vwgt"][:nc], bufs["nwgt"][:mc])
    return cid, H


def project(cid, coarse_part):
    torch = _torch()
    part = torch.empty(cid.numel(), dtype=torch.int32, device=cid.device)
    _check(lib().hgp_project(cid.numel(), _ptr(cid), _ptr(coarse_part), _ptr(part), _stream()), "hgp_project")
    return part


def objective(h: Hypergraph, k: int, part):
    torch = _torch()
    f = torch.zeros(1, dtype=torch.int64, device=h.device)
    bw = torch.zeros(k, dtype=torch.int64, device=h.device)
    ws = _ws(OP_REFINE, h, params(k))
    s = h.struct()
    _check(lib().hgp_objective(ctypes.byref(s), k, _ptr(part), _ptr(f), _ptr(bw), _ptr(ws), ws.numel(),
                               _stream()), "hgp_objective")
    return int(f.item()), bw


def refine_lp(h: Hypergraph, prm: Params, level: int, part):
    """LP refinement in place on `part`; returns (objective, block weights)."""
    torch = _torch()
    f = torch.zeros(1, dtype=torch.int64, device=h.device)
    bw = torch.zeros(prm.k, dtype=torch.int64, device=h.device)
    ws = _ws(OP_REFINE, h, prm)
    s = h.struct()
    _check(lib().hgp_refine_lp(ctypes.byref(s), ctypes.byref(prm), level, _ptr(part), _ptr(f), _ptr(bw),
                               _ptr(ws), ws.numel(), _stream()), "hgp_refine_lp")
    return int(f.item()), bw


def gain_table(h: Hypergraph, k: int, part, ws=None):
    """hgp_gain_table: (benefit int32 [n], penalty int32 [n, k])."""
    torch = _torch()
    ben = torch.empty(h.n, dtype=torch.int32, device=h.device)
    pen = torch.empty((h.n, k), dtype=torch.int32, device=h.device)
    ws = _ws(OP_GAINS, h, params(k)) if ws is None else ws
    s = h.struct()
    _check(lib().hgp_gain_table(ctypes.byref(s), k, _ptr(part), _ptr(ben), _ptr(pen), _ptr(ws), ws.numel(),
                                _stream()), "hgp_gain_table")
    return ben, pen


def gain_table_update(h: Hypergraph, k: int, part, node, target, ben, pen, ws=None):
    """hgp_gain_table_update: applies the moves to part and updates the
    table in place."""
    ws = _ws(OP_GAINS, h, params(k)) if ws is None else ws
    s = h.struct()
    _check(lib().hgp_gain_table_update(ctypes.byref(s), k, _ptr(part), _ptr(node), _ptr(target), node.numel(),
                                       _ptr(ben), _ptr(pen), _ptr(ws), ws.numel(), _stream()),
           "hgp_gain_table_update")


def gain_recalc(h: Hypergraph, k: int, part, node, target, ws=None):
    """hgp_gain_recalc: int64 gain of every move of the sequence."""
    torch = _torch()
    g = torch.empty(max(node.numel(), 1), dtype=torch.int64, device=h.device)
    ws = _ws(OP_GAINS, h, params(k)) if ws is None else ws
    s = h.struct()
    _check(lib().hgp_gain_recalc(ctypes.byref(s), k, _ptr(part), _ptr(node), _ptr(target), node.numel(), _ptr(g),
                                 _ptr(ws), ws.numel(), _stream()), "hgp_gain_recalc")
    return g[:node.numel()]


def communities(h: Hypergraph, seed: int = 0, ws=None):
    """hgp_communities: (community id per vertex (int32 tensor), Louvain levels)."""
    torch = _torch()
    comm = torch.empty(h.n, dtype=torch.int32, device=h.device)
    ws = _ws(OP_COMMUNITY, h, params(2)) if ws is None else ws
    lv = ctypes.c_uint32(0)
    s = h.struct()
    _check(lib().hgp_communities(ctypes.byref(s), seed, _ptr(comm), ctypes.byref(lv), _ptr(ws), ws.numel(),
                                 _stream()), "hgp_communities")
    return comm, int(lv.value)


def graph_gain_table(h: Hypergraph, k: int, part, ws=None):
    """hgp_graph_gain_table: omega int32 [n, k] = w(u, V_i) of a graph."""
    torch = _torch()
    om = torch.empty((h.n, k), dtype=torch.int32, device=h.device)
    ws = _ws(OP_GAINS, h, params(k)) if ws is None else ws
    s = h.struct()
    _check(lib().hgp_graph_gain_table(ctypes.byref(s), k, _ptr(part), _ptr(om), _ptr(ws), ws.numel(), _stream()),
           "hgp_graph_gain_table")
    return om


def graph_moves(h: Hypergraph, k: int, part, node, target, omega=None, gains=True, ws=None):
    """hgp_graph_moves: applies the moves to part, updates omega in place
    when given, and returns the int64 attributed gains (or None)."""
    torch = _torch()
    g = torch.empty(max(node.numel(), 1), dtype=torch.int64, device=h.device) if gains else None
    ws = _ws(OP_GAINS, h, params(k)) if ws is None else ws
    s = h.struct()
    _check(lib().hgp_graph_moves(ctypes.byref(s), k, _ptr(part), _ptr(node), _ptr(target), node.numel(),
                                 _ptr(omega) if omega is not None else None, _ptr(g) if g is not None else None,
                                 _ptr(ws), ws.numel(), _stream()), "hgp_graph_moves")
    return g[:node.numel()] if g is not None else None


STATIC_SCRATCH_BYTES = 64 << 20  # HGP_STATIC_SCRATCH_BYTES


def refine_lp_static(h: Hypergraph, prm: Params, level: int, part):
    """hgp_refine_lp_static: the same refinement with the library's fixed
    device scratch array (no workspace); returns (objective, block weights)."""
    torch = _torch()
    f = torch.zeros(1, dtype=torch.int64, device=h.device)
    bw = torch.zeros(prm.k, dtype=torch.int64, device=h.device)
    s = h.struct()
    _check(lib().hgp_refine_lp_static(ctypes.byref(s), ctypes.byref(prm), level, _ptr(part), _ptr(f), _ptr(bw),
                                      _stream()), "hgp_refine_lp_static")
    return int(f.item()), bw


def initial_partition(h: Hypergraph, k: int):
    torch = _torch()
    part = torch.empty(h.n, dtype=torch.int32, device=h.device)
    ws = _ws(OP_INITIAL, h, params(k))
    s = h.struct()
    _check(lib().hgp_initial_partition(ctypes.byref(s), k, _ptr(part), _ptr(ws), ws.numel(), _stream()),
           "hgp_initial_partition")
    return part


def rb_initial_partition(h: Hypergraph, prm: Params, ws=None):
    """hgp_rb_initial_partition: the recursive-bipartitioning initial
    partition (Sec. 5, Eq. 1) of h into prm.k blocks (int32 tensor)."""
    torch = _torch()
    part = torch.empty(h.n, dtype=torch.int32, device=h.device)
    ws = _ws(OP_RB, h, prm) if ws is None else ws
    s = h.struct()
    _check(lib().hgp_rb_initial_partition(ctypes.byref(s), ctypes.byref(prm), _ptr(part), _ptr(ws), ws.numel(),
                                          _stream()), "hgp_rb_initial_partition")
    return part


class Partitioner:
    """Reusable partitioner: the workspace is allocated once per size."""

    def __init__(self, h: Hypergraph, prm: Params, ws=None):
        torch = _torch()
        self.h, self.prm = h, prm
        self.ws = _ws(OP_PARTITION, h, prm) if ws is None else ws
        self.part = torch.empty(h.n, dtype=torch.int32, device=h.device)
        self.f = torch.zeros(1, dtype=torch.int64, device=h.device)
        self._s = h.struct()

    def run(self):
        lv = ctypes.c_uint32(0)
        _check(lib().hgp_partition(ctypes.byref(self._s), ctypes.byref(self.prm), _ptr(self.part), _ptr(self.f),
                                   ctypes.byref(lv), _ptr(self.ws), self.ws.numel(), _stream()), "hgp_partition")
        return int(lv.value)


    def run_traced(self, cap: int = 256):
        """One run through hgp_partition_traced; returns a list of per-level
        dicts (n, m, p, lp_rounds), level 0 first."""
        arr = {f: np.zeros(cap, np.uint32) for f in ("n", "m", "p", "lp_rounds")}
        tr = _Trace(cap, 0, *[arr[f].ctypes.data for f in ("n", "m", "p", "lp_rounds")])
        _check(lib().hgp_partition_traced(ctypes.byref(self._s), ctypes.byref(self.prm), _ptr(self.part),
                                          _ptr(self.f), ctypes.byref(tr), _ptr(self.ws), self.ws.numel(),
                                          _stream()), "hgp_partition_traced")
        L = min(int(tr.levels) + 1, cap)
        return [{f: int(arr[f][l]) for f in arr} for l in range(L)]


def partition(h: Hypergraph, prm: Params):
    """Whole multilevel partition; returns (part tensor, objective, levels)."""
    P = Partitioner(h, prm)
    levels = P.run()
    return P.part, int(P.f.item()), levels


class KernelTimer:
    """Per-kernel measurement through the library's event timing and
    compulsory-byte accounting (see hgp_timing_begin)."""

    def __init__(self, n_max: int, m_max: int, device="cuda"):
        torch = _torch()
        nb = ctypes.c_size_t(0)
        _check(lib().hgp_timing_scratch_bytes(n_max, m_max, ctypes.byref(nb)), "hgp_timing_scratch_bytes")
        self.scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.n_max, self.m_max = n_max, m_max

    def begin(self, mask: int, account: bool = False):
        _check(lib().hgp_timing_begin(mask, int(account), _ptr(self.scratch), self.scratch.numel(), self.n_max,
                                      self.m_max), "hgp_timing_begin")

    def sample(self, every: int, phase: int):
        """Events on launch j of each timed kernel only when j % every == phase
        (counted from this call; see hgp_timing_sample)."""
        _check(lib().hgp_timing_sample(every, phase), "hgp_timing_sample")

    def end(self):
        k = len(KERNELS)
        ms = (ctypes.c_double * k)()
        ln = (ctypes.c_uint64 * k)()
        by = (ctypes.c_double * k)()
        _check(lib().hgp_timing_end(k, ms, ln, by), "hgp_timing_end")
        return [dict(kernel=KERNELS[i], ms=ms[i], launches=int(ln[i]), bytes=by[i]) for i in range(k)]


def partition_batch(hs, prms, lanes: int = 8, ws_bytes: int | None = None):
    """Partitions the Hypergraphs hs[i] with Params prms[i] in one batch call
    (hgp_partition_batch).  Returns (list of part tensors, objectives (int64
    tensor), levels list)."""
    torch = _torch()
    count = len(hs)
    HG = _HG * count
    PA = Params * count
    structs = HG(*[h.struct() for h in hs])
    params_ = PA(*prms)
    need = ctypes.c_size_t(0)
    _check(lib().hgp_batch_workspace_bytes(structs, params_, count, lanes, ctypes.byref(need)),
           "hgp_batch_workspace_bytes")
    nb = int(need.value) if ws_bytes is None else int(ws_bytes)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=hs[0].device)
    parts = [torch.empty(h.n, dtype=torch.int32, device=h.device) for h in hs]
    pptr = (ctypes.c_void_p * count)(*[p.data_ptr() for p in parts])
    objs = torch.zeros(count, dtype=torch.int64, device=hs[0].device)
    lv = (ctypes.c_uint32 * count)()
    _check(lib().hgp_partition_batch(structs, params_, count, lanes, pptr, _ptr(objs), lv, _ptr(ws), ws.numel(),
                                     _stream()), "hgp_partition_batch")
    return parts, objs, list(lv)


class Server:
    """Continuous-admission partition server (hgp_server_*): requests are
    admitted as lanes and pool memory free up and run overlapped."""

    def __init__(self, lanes: int, pool_bytes: int, device="cuda"):
        torch = _torch()
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=device)
        self._h = ctypes.c_void_p(0)
        _check(lib().hgp_server_create(lanes, _ptr(self.pool), self.pool.numel(), ctypes.byref(self._h)),
               "hgp_server_create")
        self._live = {}

    def submit(self, h: Hypergraph, prm: Params):
        """Queues one request; returns (ticket, part tensor, objective tensor)."""
        torch = _torch()
        part = torch.empty(h.n, dtype=torch.int32, device=h.device)
        obj = torch.zeros(1, dtype=torch.int64, device=h.device)
        s = h.struct()
        p = Params(prm.k, prm.eps_num, prm.eps_den, prm.seed, prm.limit_factor, prm.coarsen_subrounds,
                   prm.lp_subrounds, prm.lp_rounds, prm.flags)
        t = ctypes.c_uint64(0)
        _check(lib().hgp_server_submit(self._h, ctypes.byref(s), ctypes.byref(p), _ptr(part), _ptr(obj), _stream(),
                                       ctypes.byref(t)), "hgp_server_submit")
        self._live[t.value] = (h, part, obj)  # keep the inputs alive until the wait
        return t.value, part, obj

    def wait(self, ticket: int):
        """Blocks until the request is done; returns (levels, latency_ms, queue_ms)."""
        lv = ctypes.c_uint32(0)
        lat = ctypes.c_double(0)
        qm = ctypes.c_double(0)
        st = lib().hgp_server_wait(self._h, ticket, ctypes.byref(lv), ctypes.byref(lat), ctypes.byref(qm))
        self._live.pop(ticket, None)
        _check(st, "hgp_server_wait")
        return int(lv.value), lat.value, qm.value

    def close(self):
        if self._h:
            lib().hgp_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
