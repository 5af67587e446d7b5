"""Pure-Python brute force from the paper's definitions, on tiny inputs.

Independent of the oracle: sets and dictionaries, no shared code.  Used to pin
the oracle (and through it the GPU path)."""
from __future__ import annotations

import itertools


def nets_of(h):
    return [tuple(int(x) for x in h.pins[h.pin_off[e]:h.pin_off[e + 1]]) for e in range(h.m)]


def objective(h, part):
    """Connectivity metric: sum over cut nets of (lambda(e) - 1) * w(e)."""
    f = 0
    for e, pins in enumerate(nets_of(h)):
        lam = len({int(part[v]) for v in pins})
        if lam > 1:
            f += (lam - 1) * int(h.nwgt[e])
    return f


def cut_net(h, part):
    """Cut-net metric: total weight of nets spanning more than one block."""
    return sum(int(h.nwgt[e]) for e, pins in enumerate(nets_of(h)) if len({int(part[v]) for v in pins}) > 1)


def move_delta(h, part, u, t):
    """f(Pi) - f(Pi with u moved to t), recomputed from scratch."""
    q = [int(x) for x in part]
    before = objective(h, q)
    q[u] = t
    return before - objective(h, q)


def rating(h, rep, u):
    """r(u, C) = sum over nets e with u in e and e touching C of floor(w * 2^32 / (|e|-1));
    C ranges over clusters other than u's, identified by representative."""
    members = {}
    for v, c in enumerate(rep):
        members.setdefault(int(c), set()).add(v)
    nets = nets_of(h)
    R = {}
    for C, mem in members.items():
        if C == int(rep[u]):
            continue
        tot = 0
        for e, pins in enumerate(nets):
            if len(pins) >= 2 and u in pins and mem.intersection(pins):
                tot += (int(h.nwgt[e]) << 32) // (len(pins) - 1)
        if tot:
            R[C] = tot
    return R


def contract_sets(h, rep):
    """Contraction by sets: coarse net multiset {frozenset(cluster ids): summed weight}
    with single-pin nets removed; clusters named by their representative."""
    out = {}
    for e, pins in enumerate(nets_of(h)):
        s = frozenset(int(rep[v]) for v in pins)
        if len(s) < 2:
            continue
        out[s] = out.get(s, 0) + int(h.nwgt[e])
    return out


def merge_path_states(ca, cb):
    """States (i, j) of merging the exclusive prefix sums of A and B by value,
    A first on ties -- the merge reading of the two-pointer walk."""
    pa = list(itertools.accumulate([0] + list(ca)))[:-1]
    pb = list(itertools.accumulate([0] + list(cb)))[:-1]
    items = [(pa[i], 0, i) for i in range(len(ca))] + [(pb[j], 1, j) for j in range(len(cb))]
    items.sort()
    states = [(0, 0)]
    i = j = 0
    for _, side, _idx in items:
        if side == 0:
            i += 1
        else:
            j += 1
        states.append((i, j))
    return states


# ---------------------------------------------------------------------------
# Seeded hash from its definition, independent of the oracle's C code.
# mix64 is the SplitMix64 finalizer (Steele, Lea, Flood 2014); the tests pin
# it to the published outputs of that generator.  The tag layout is the one
# fixed for this method's determinism: H(seed, purpose, level, it, x) =
# mix64(mix64(seed) XOR ((purpose | level << 8 | it << 16) << 32 | x)), with
# purpose 1 = coarsening sub-round, 2 = rating tie, 3 = LP sub-round.
# ---------------------------------------------------------------------------
M64 = (1 << 64) - 1


def mix64(z):
    z &= M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def H(seed, purpose, level, it, x):
    tag = (purpose & 0xFF) | ((level & 0xFF) << 8) | ((it & 0xFFFF) << 16)
    return mix64(mix64(seed) ^ ((tag << 32) | (x & 0xFFFFFFFF)))


# ---------------------------------------------------------------------------
# Gain table and move-sequence gains (Sec. 6.2, 6.3) from the definitions
# ---------------------------------------------------------------------------
def phi(h, part, e, b):
    return sum(1 for v in nets_of(h)[e] if int(part[v]) == b)


def gain_table(h, k, part):
    """benefit b(u) = w(nets of u where u is the only pin of its block) and
    penalty p(u, t) = w(nets of u with no pin in block t)."""
    nets = nets_of(h)
    ben = [0] * h.n
    pen = [[0] * k for _ in range(h.n)]
    for e, pins in enumerate(nets):
        w = int(h.nwgt[e])
        blocks = [int(part[v]) for v in pins]
        for v in pins:
            if blocks.count(int(part[v])) == 1:
                ben[v] += w
            for t in range(k):
                if t not in blocks:
                    pen[v][t] += w
    return ben, pen


def sequence_gains(h, part, moves):
    """Objective decrease of each move when the moves are performed in order."""
    q = [int(x) for x in part]
    out = []
    for u, t in moves:
        before = objective(h, q)
        q[u] = t
        out.append(before - objective(h, q))
    return out


def alg4_gains(h, part, moves):
    """The paper's parallel gain recalculation (Sec. 6.3), one net at a time:
    for every block, the index of the first move into it and of the last move
    out of it among the net's pins, and the number of unmoved pins in it; a
    move gains w(e) when it is the last to leave a block that ends empty of
    unmoved pins before any pin arrives, and loses w(e) when it is the first to
    arrive in a block left empty in that way earlier."""
    idx = {u: i for i, (u, t) in enumerate(moves)}
    g = [0] * len(moves)
    for e, pins in enumerate(nets_of(h)):
        w = int(h.nwgt[e])
        first_in, last_out, unmoved = {}, {}, {}
        for v in pins:
            if v in idx:
                i = idx[v]
                s, t = int(part[v]), moves[i][1]
                last_out[s] = max(i, last_out.get(s, -1))
                first_in[t] = min(i, first_in.get(t, len(moves)))
            else:
                b = int(part[v])
                unmoved[b] = unmoved.get(b, 0) + 1
        for v in pins:
            if v not in idx:
                continue
            i = idx[v]
            s, t = int(part[v]), moves[i][1]
            if last_out.get(s) == i and i < first_in.get(s, len(moves)) and unmoved.get(s, 0) == 0:
                g[i] += w
            if first_in.get(t) == i and i > last_out.get(t, -1) and unmoved.get(t, 0) == 0:
                g[i] -= w
    return g


# ---------------------------------------------------------------------------
# Community detection (Sec. 4.3): bipartite graph and modularity
# ---------------------------------------------------------------------------
def bipartite_edges(h):
    """Edges {u, n + e} of the bipartite graph, one per pin, with weight w(e)."""
    out = []
    for e, pins in enumerate(nets_of(h)):
        for u in pins:
            out.append((u, h.n + e, int(h.nwgt[e])))
    return out


def modularity(edges, comm):
    """Q = sum over communities C of in(C) / M - (vol(C) / 2M)^2, exactly (Fraction);
    edges is a list of (a, b, w) with a != b, M the total edge weight."""
    from fractions import Fraction
    M = sum(w for _, _, w in edges)
    inw, vol = {}, {}
    for a, b, w in edges:
        vol[comm[a]] = vol.get(comm[a], 0) + w
        vol[comm[b]] = vol.get(comm[b], 0) + w
        if comm[a] == comm[b]:
            inw[comm[a]] = inw.get(comm[a], 0) + w
    return sum(Fraction(inw.get(c, 0), M) - Fraction(v, 2 * M) ** 2 for c, v in vol.items())


def louvain_subround(edges, n_nodes, comm, seed, level, r, s, S=5):
    """One synchronous local-moving sub-round from the definition: each node of
    the sub-round takes the neighbour community that raises Q the most (ties:
    smaller ID) if it raises Q at all, judged on the state at the start; then
    all moves are made."""
    adj = [[] for _ in range(n_nodes)]
    for a, b, w in edges:
        adj[a].append(b)
        adj[b].append(a)
    q0 = modularity(edges, comm)
    dec = {}
    for x in range(n_nodes):
        if H(seed, 4, level, r, x) % S != s:
            continue
        best, best_d = None, None
        for c in sorted({comm[y] for y in adj[x]} - {comm[x]}):
            trial = list(comm)
            trial[x] = c
            d = modularity(edges, trial) - q0
            if best is None or d > best_d:
                best, best_d = c, d
        if best is not None and best_d > 0:
            dec[x] = best
    out = list(comm)
    for x, c in dec.items():
        out[x] = c
    return out, len(dec)
