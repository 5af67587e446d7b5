"""Seeded synthetic hypergraph generators and the host-side CSR container.

This module only builds inputs: it holds none of the partitioning method's
arithmetic, so both the GPU library's tests and the CPU oracle can use it.

Every instance is a set of nets over vertices 0..n-1, stored as two CSR
adjacency arrays (pins per net, incident nets per vertex), which is the
hypergraph layout of Sec. 4.2 of the paper.  Pins are strictly ascending
inside each net and nets ascending inside each incidence list.

Random draws use a counter-based generator (no hidden state):
    r(seed, stream, i) = mix64(mix64(seed) ^ (stream << 40) ^ i)
with mix64 the SplitMix64 finalizer, and uniform(N) = (r * N) >> 64.
The paper's own benchmark sets are not available; these generators stand in
for them with the shapes and distributions of the workloads named below.
"""
from __future__ import annotations

import dataclasses
import numpy as np

U64 = np.uint64
_M1 = U64(0xBF58476D1CE4E5B9)
_M2 = U64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=U64).copy()
    z ^= z >> U64(30)
    z *= _M1
    z ^= z >> U64(27)
    z *= _M2
    z ^= z >> U64(31)
    return z


def rng(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """64-bit counter-based draws for counters idx of one stream."""
    base = _mix64(np.array([seed & (2**64 - 1)], dtype=U64))[0]
    key = base ^ U64((stream << 40) & (2**64 - 1))
    return _mix64(np.asarray(idx, dtype=U64) ^ key)


def uniform(r: np.ndarray, bound) -> np.ndarray:
    """floor(r * bound / 2^64) for bound < 2^32 (elementwise bound allowed)."""
    r = np.asarray(r, dtype=U64)
    b = np.asarray(bound, dtype=U64)
    hi = r >> U64(32)
    lo = r & U64(0xFFFFFFFF)
    return ((hi * b) + ((lo * b) >> U64(32))) >> U64(32)


def uniform64(r: np.ndarray, bound: int) -> np.ndarray:
    """floor(r * bound / 2^64) for bound < 2^63, exact (Python big ints in chunks)."""
    r = np.asarray(r, dtype=U64)
    if bound < 2**32:
        return uniform(r, bound)
    bh, bl = U64(bound >> 32), U64(bound & 0xFFFFFFFF)
    rh, rl = r >> U64(32), r & U64(0xFFFFFFFF)
    # (rh*2^32 + rl) * (bh*2^32 + bl) >> 64
    hh = rh * bh
    hl = rh * bl
    lh = rl * bh
    ll = rl * bl
    mid = (hl & U64(0xFFFFFFFF)) + (lh & U64(0xFFFFFFFF)) + (ll >> U64(32))
    return hh + (hl >> U64(32)) + (lh >> U64(32)) + (mid >> U64(32))


@dataclasses.dataclass
class HostHypergraph:
    """Hypergraph in host memory (numpy).  IDs and offsets uint32, weights int32."""

    n: int
    m: int
    pin_off: np.ndarray
    pins: np.ndarray
    inc_off: np.ndarray
    inc: np.ndarray
    vwgt: np.ndarray
    nwgt: np.ndarray
    name: str = ""

    @property
    def p(self) -> int:
        return int(self.pins.shape[0])

    def net(self, e: int) -> np.ndarray:
        return self.pins[self.pin_off[e]:self.pin_off[e + 1]]

    def incident(self, v: int) -> np.ndarray:
        return self.inc[self.inc_off[v]:self.inc_off[v + 1]]


def _stable_argsort(keys: np.ndarray) -> np.ndarray:
    """Stable argsort of an integer array.  Large arrays go through torch's
    multithreaded CPU radix sort (same permutation: a stable order is unique)."""
    if keys.size < (1 << 22):
        return np.argsort(keys, kind="stable")
    import torch
    _, idx = torch.sort(torch.from_numpy(np.ascontiguousarray(keys).astype(np.int64)), stable=True)
    return idx.numpy()


def _workers() -> int:
    import os
    return max(1, min(16, os.cpu_count() or 1))


def transpose(n: int, m: int, pin_off: np.ndarray, pins: np.ndarray):
    """Incidence CSR (nets ascending per vertex) from the pin CSR."""
    sizes = np.diff(pin_off.astype(np.int64))
    net_of_pin = np.repeat(np.arange(m, dtype=np.uint32), sizes)
    order = _stable_argsort(pins)
    inc = net_of_pin[order].astype(np.uint32)
    del order, net_of_pin
    deg = np.bincount(pins.astype(np.int64), minlength=n).astype(np.int64)
    inc_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=inc_off[1:])
    return inc_off.astype(np.uint32), inc


def from_nets(n: int, nets, vwgt=None, nwgt=None, name: str = "") -> HostHypergraph:
    """Build from a list of pin lists (each is sorted and de-duplicated)."""
    lists = [np.unique(np.asarray(e, dtype=np.int64)) for e in nets]
    m = len(lists)
    sizes = np.array([len(e) for e in lists], dtype=np.int64)
    pin_off = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=pin_off[1:])
    pins = (np.concatenate(lists) if m and pin_off[-1] else np.zeros(0, np.int64)).astype(np.uint32)
    if pins.size and (pins.max() >= n):
        raise ValueError("pin out of range")
    pin_off = pin_off.astype(np.uint32)
    inc_off, inc = transpose(n, m, pin_off, pins)
    vw = np.ones(n, np.int32) if vwgt is None else np.asarray(vwgt, np.int32)
    nw = np.ones(m, np.int32) if nwgt is None else np.asarray(nwgt, np.int32)
    return HostHypergraph(n, m, pin_off, pins, inc_off, inc, vw, nw, name)


def _finish(n, m, sizes, pins_sorted, vwgt, nwgt, name) -> HostHypergraph:
    pin_off = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes.astype(np.int64), out=pin_off[1:])
    pin_off = pin_off.astype(np.uint32)
    pins = pins_sorted.astype(np.uint32)
    inc_off, inc = transpose(n, m, pin_off, pins)
    return HostHypergraph(n, m, pin_off, pins, inc_off, inc,
                          np.asarray(vwgt, np.int32), np.asarray(nwgt, np.int32), name)


def _draw_distinct_pins(seed: int, first_stream: int, n: int, sizes: np.ndarray, draw, with_net: bool = False):
    """Pins of every net drawn independently, redrawing repeats inside a net.

    Slot q (global pin position) on attempt a uses counter q of stream
    first_stream + a.  The earliest slot holding a value keeps it; later
    slots with the same value in the same net are redrawn.  Returns pins
    sorted ascending inside every net."""
    m = sizes.shape[0]
    total = int(sizes.sum())
    net = np.repeat(np.arange(m, dtype=np.int64), sizes.astype(np.int64))
    slots = np.arange(total, dtype=np.int64)
    if with_net:
        base_draw = draw
        draw = None

        def draw_at(r, idx):
            return base_draw(r, net[idx])
    else:
        def draw_at(r, idx):
            return draw(r)
    vals = draw_at(rng(seed, first_stream, slots), slots)
    attempt = 0
    redo = None
    assert n < 2**32 and m < 2**31
    while True:
        # by net, then value, then slot (a stable sort keeps slot order)
        order = np.argsort((net << 32) | vals, kind="stable")
        key = ((net << 32) | vals)[order]
        dup = np.zeros(total, dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        redo = order[dup]
        if redo.size == 0:
            break
        attempt += 1
        if attempt > 10000:
            raise RuntimeError("pin redraw did not converge (net larger than the vertex pool?)")
        vals[redo] = draw_at(rng(seed, first_stream + attempt, redo), redo)
    return vals[np.argsort((net << 32) | vals, kind="stable")]


def random_uniform(n: int = 10_000, m: int = 10_000, smin: int = 2, smax: int = 8,
                   seed: int = 1, name: str = "random") -> HostHypergraph:
    """Random hypergraph: net sizes uniform in [smin, smax], pins uniform
    without replacement, unit weights (small plain-method workload)."""
    sizes = smin + uniform(rng(seed, 0, np.arange(m)), smax - smin + 1).astype(np.int64)
    pins = _draw_distinct_pins(seed, 1, n, sizes, lambda r: uniform(r, n).astype(np.int64))
    return _finish(n, m, sizes, pins, np.ones(n, np.int32), np.ones(m, np.int32), name)


def _zipf_table(alpha: float, lo: int, hi: int) -> np.ndarray:
    """Integer inverse-CDF thresholds (53-bit) of P(s) ~ s^-alpha on [lo, hi]."""
    s = np.arange(lo, hi + 1, dtype=np.float64)
    w = s ** (-alpha)
    c = np.cumsum(w)
    thr = np.floor(c / c[-1] * float(2**53)).astype(np.int64)
    thr[-1] = 2**53
    return thr


def _zipf_draw(r: np.ndarray, thr: np.ndarray, lo: int) -> np.ndarray:
    u = (np.asarray(r, dtype=U64) >> U64(11)).astype(np.int64)
    return lo + np.searchsorted(thr, u, side="right").astype(np.int64)


def powerlaw(n: int = 1_000_000, m: int = 1_000_000, alpha_size: float = 2.1,
             max_size: int = 1000, alpha_deg: float = 2.3, max_w: int = 4,
             seed: int = 2, name: str = "powerlaw") -> HostHypergraph:
    """Power-law hypergraph: net sizes Zipf(alpha_size) on [2, max_size];
    vertex sampling weights iid Zipf(alpha_deg) on [1, n] (power-law vertex
    degrees); pins drawn proportionally to those weights without replacement;
    net weights uniform in [1, max_w]; unit vertex weights."""
    max_size = min(max_size, n)
    sizes = _zipf_draw(rng(seed, 0, np.arange(m)), _zipf_table(alpha_size, 2, max_size), 2)
    dw = _zipf_draw(rng(seed, 1, np.arange(n)), _zipf_table(alpha_deg, 1, n), 1)
    cum = np.cumsum(dw.astype(np.int64))
    tot = int(cum[-1])

    def draw(r):
        x = uniform64(r, tot).astype(np.int64)
        return np.searchsorted(cum, x, side="right").astype(np.int64)

    pins = _draw_distinct_pins(seed, 3, n, sizes, draw)
    nw = 1 + uniform(rng(seed, 2, np.arange(m)), max_w).astype(np.int32)
    return _finish(n, m, sizes, pins, np.ones(n, np.int32), nw, name)


def stencil3d(N: int = 160, name: str = "") -> HostHypergraph:
    """Row-net model of a 3D 7-point stencil on an N^3 grid: vertex id
    x + N(y + N z); net j = {j} plus its in-grid axis neighbours (size 4..7);
    unit weights; no randomness."""
    n = N * N * N
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    cols = []
    masks = []
    for dx, dy, dz in ((0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)):
        ok = (x + dx >= 0) & (x + dx < N) & (y + dy >= 0) & (y + dy < N) & (z + dz >= 0) & (z + dz < N)
        cols.append(idx + dx + N * (dy + N * dz))
        masks.append(ok)
    C = np.stack(cols, axis=1)  # ascending by construction (offsets ordered)
    Mk = np.stack(masks, axis=1)
    sizes = Mk.sum(axis=1)
    pins = C[Mk]
    return _finish(n, n, sizes, pins, np.ones(n, np.int32), np.ones(n, np.int32),
                   name or f"stencil{N}")


def rmat(scale: int = 24, edges: int = 2**28, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 3, chunk: int = 1 << 22, name: str = "") -> HostHypergraph:
    """R-MAT graph as a hypergraph of 2-pin nets (one net per edge).

    Edge i, recursion level l, attempt t draws 32 bits from counter
    (i * scale + l) of stream 1 + t (upper or lower half of the 64-bit draw for
    even/odd l).  Quadrant thresholds are integers floor(p * 2^32).  Self
    loops are redrawn (next attempt); duplicate edges are kept.  Vertex IDs are
    relabelled by the permutation that sorts mix64(seed-keyed id)."""
    n = 1 << scale
    ta = int(a * 2**32)
    tb = int((a + b) * 2**32)
    tc = int((a + b + c) * 2**32)
    src = np.empty(edges, dtype=np.int64)
    dst = np.empty(edges, dtype=np.int64)

    def gen(ids, attempt):
        s = np.zeros(ids.size, dtype=np.int64)
        d = np.zeros(ids.size, dtype=np.int64)
        for l in range(0, scale, 2):
            r = rng(seed, 1 + attempt, ids.astype(U64) * U64(scale) + U64(l))
            for half in (0, 1):
                if l + half >= scale:
                    break
                v = ((r >> U64(32)) if half == 0 else (r & U64(0xFFFFFFFF))).astype(np.int64)
                sb = (v >= tb).astype(np.int64)
                db = (((v >= ta) & (v < tb)) | (v >= tc)).astype(np.int64)
                s = s * 2 + sb
                d = d * 2 + db
        return s, d

    def fill(lo):
        ids = np.arange(lo, min(edges, lo + chunk), dtype=np.int64)
        s, d = gen(ids, 0)
        attempt = 0
        bad = np.nonzero(s == d)[0]
        while bad.size:
            attempt += 1
            s2, d2 = gen(ids[bad], attempt)
            s[bad], d[bad] = s2, d2
            bad = bad[s2 == d2]
        src[lo:lo + ids.size] = s
        dst[lo:lo + ids.size] = d

    # chunks are independent (counter-based draws); numpy releases the GIL in
    # its element-wise loops, so threads run them in parallel
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill, range(0, edges, chunk)))
    perm_key = rng(seed, 0, np.arange(n))
    order = np.argsort(perm_key, kind="stable")
    relabel = np.empty(n, dtype=np.int64)
    relabel[order] = np.arange(n, dtype=np.int64)
    s = relabel[src]
    d = relabel[dst]
    del src, dst
    lo_ = np.minimum(s, d)
    hi_ = np.maximum(s, d)
    del s, d
    pins = np.empty(2 * edges, dtype=np.uint32)
    pins[0::2] = lo_
    pins[1::2] = hi_
    del lo_, hi_
    sizes = np.full(edges, 2, dtype=np.int64)
    return _finish(n, edges, sizes, pins, np.ones(n, np.int32), np.ones(edges, np.int32),
                   name or f"rmat{scale}")


def _unit_real(r: np.ndarray) -> np.ndarray:
    """(r >> 11) * 2^-53 in [0, 1)."""
    return (np.asarray(r, dtype=U64) >> U64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def vlsi_params(count: int = 4096, seed: int = 4):
    """(n, k) of every instance of the batch workload: n = floor(exp(ln 1e3 +
    u ln 200)) (log-uniform on [1e3, 2e5]), k uniform in {2, 4, 8}."""
    idx = np.arange(count)
    u = _unit_real(rng(seed, 0, idx))
    n = np.floor(np.exp(np.log(1e3) + u * np.log(200.0))).astype(np.int64)
    k = np.array([2, 4, 8], dtype=np.int64)[uniform(rng(seed, 1, idx), 3).astype(np.int64)]
    return n, k


def vlsi(n: int, inst: int, seed: int = 4, name: str = "") -> HostHypergraph:
    """One VLSI-like instance of the batch workload: m = floor(1.1 n) nets of
    size 2 + Geometric(0.4) (failures before the first success, inverse CDF of
    a 53-bit uniform), capped at 50; each net has an anchor a = uniform(n) and
    each pin lies with probability 0.9 in the window of 256 IDs starting at
    clamp(a - 128, 0, n - 256), otherwise anywhere; pins distinct per net;
    vertex weights 1 + uniform(10), unit net weights.  Instance `inst` draws
    from its own seed (seed << 32 | inst)."""
    s = (seed << 32) | inst
    m = int(np.floor(1.1 * n))
    ids = np.arange(m)
    g = np.floor(np.log1p(-_unit_real(rng(s, 0, ids))) / np.log(0.6)).astype(np.int64)
    sizes = np.minimum(2 + g, 50)
    anchor = uniform(rng(s, 1, ids), n).astype(np.int64)
    w0 = np.clip(anchor - 128, 0, max(n - 256, 0))
    win = min(256, n)
    thr = U64(int(0.9 * 2**32))

    def draw(r, net_ids):
        hi = r >> U64(32)
        lo = r & U64(0xFFFFFFFF)
        local = hi < thr
        pos_local = w0[net_ids] + ((lo * U64(win)) >> U64(32)).astype(np.int64)
        pos_any = ((lo * U64(n)) >> U64(32)).astype(np.int64)
        return np.where(local, pos_local, pos_any)

    pins = _draw_distinct_pins(s, 3, n, sizes, draw, with_net=True)
    vw = 1 + uniform(rng(s, 2, np.arange(n)), 10).astype(np.int32)
    return _finish(n, m, sizes, pins, vw, np.ones(m, np.int32), name or f"vlsi{inst}")


def vlsi_batch(count: int = 4096, seed: int = 4):
    """The batch workload: list of (hypergraph, k) for instances 0..count-1."""
    ns, ks = vlsi_params(count, seed)
    return [(vlsi(int(ns[i]), i, seed), int(ks[i])) for i in range(count)]


def serve_trace(count: int = 200, seed: int = 5):
    """Requests of the serving workload: per request a target pin count
    P = floor(exp(ln 1e4 + u ln 1e3)) (log-uniform on [1e4, 1e7]), a family
    uniform over {random, power-law, stencil, R-MAT} sized to about P pins,
    and k uniform in {2..64}.  Returns a list of (family, P, k)."""
    idx = np.arange(count)
    u = _unit_real(rng(seed, 0, idx))
    P = np.floor(np.exp(np.log(1e4) + u * np.log(1e3))).astype(np.int64)
    fam = uniform(rng(seed, 1, idx), 4).astype(np.int64)
    k = 2 + uniform(rng(seed, 2, idx), 63).astype(np.int64)
    names = ("random", "powerlaw", "stencil", "rmat")
    return [(names[int(fam[i])], int(P[i]), int(k[i])) for i in range(count)]


def serve_request(family: str, P: int, j: int, seed: int = 5) -> HostHypergraph:
    """Hypergraph of one serving request (about P pins), request j's own seed."""
    s = (seed << 32) | j
    if family == "random":  # E|e| = 5
        n = max(P // 5, 16)
        return random_uniform(n, n, 2, 8, seed=s, name=f"req{j}")
    if family == "powerlaw":  # E|e| about 8.2
        n = max(P // 8, 64)
        return powerlaw(n, n, seed=s, max_size=min(1000, n // 10), name=f"req{j}")
    if family == "stencil":
        return stencil3d(max(int(round((P / 7.0) ** (1.0 / 3.0))), 3), name=f"req{j}")
    sc = max(int(round(np.log2(max(P, 64) / 32.0))), 5)  # edge factor 16, two pins per edge
    return rmat(sc, 16 << sc, seed=s, name=f"req{j}")


# Named workloads ----------------------------------------------------------
def workload(name: str) -> tuple[HostHypergraph, int]:
    """(hypergraph, k) of a named workload."""
    if name == "random10k":
        return random_uniform(10_000, 10_000, 2, 8, seed=1, name=name), 2
    if name == "powerlaw1m":
        return powerlaw(seed=2, name=name), 8
    if name == "stencil160":
        return stencil3d(160, name=name), 64
    if name == "rmat24":
        return rmat(24, 2**28, seed=3, name=name), 128
    if name.startswith("rmat"):  # e.g. rmat16: edge factor 16
        sc = int(name[len("rmat"):])
        return rmat(sc, 16 << sc, seed=3, name=name), 128
    if name.startswith("stencil"):
        return stencil3d(int(name[len("stencil"):]), name=name), 64
    if name.startswith("powerlaw"):  # e.g. powerlaw50000
        N = int(name[len("powerlaw"):])
        return powerlaw(N, N, seed=2, max_size=min(1000, N // 10), name=name), 8
    raise KeyError(name)


def move_sequence(n: int, k: int, part: np.ndarray, count: int, seed: int):
    """`count` distinct nodes in a seeded random order, each with a target
    block drawn uniformly from the k - 1 blocks other than its own: the
    shape of one round of node moves (every node moved at most once)."""
    keys = rng(seed, 1, np.arange(n))
    nodes = np.argsort(keys, kind="stable")[:count].astype(np.uint32)
    step = uniform(rng(seed, 2, np.arange(count)), k - 1).astype(np.int64) + 1
    targets = ((part[nodes].astype(np.int64) + step) % k).astype(np.uint32)
    return nodes, targets
