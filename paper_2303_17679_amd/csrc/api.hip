// extern "C" entry points: argument checks, workspace arena, the multilevel
// driver (paper Alg. 1 with the deterministic components, no FM / flows).
#include "kernels.h"
#include "timing.h"
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

using namespace hgp;

namespace {

hipStream_t S(void *stream) { return (hipStream_t)stream; }

hgp_status check_params(const hgp_params *p) {
    if (!p) return HGP_E_INVALID;
    if (p->k < 2) return HGP_E_INVALID;
    if (p->k > 256) return HGP_E_UNSUPPORTED;
    if (p->eps_den == 0 || p->eps_den > (1u << 20) || p->eps_num > p->eps_den) return HGP_E_INVALID;
    if (p->limit_factor == 0 || p->limit_factor > (1u << 20)) return HGP_E_INVALID;
    if (p->coarsen_subrounds == 0 || p->lp_subrounds == 0) return HGP_E_INVALID;
    if (p->coarsen_subrounds > 256 || p->lp_subrounds > 256 || p->lp_rounds > 65535) return HGP_E_INVALID;
    if (p->flags & ~HGP_TRUSTED_INPUT) return HGP_E_INVALID;
    if (p->community > 1 || p->ip > 1) return HGP_E_INVALID;
    return HGP_OK;
}

hgp_status check_hg(const hgp_hg *h) {
    if (!h) return HGP_E_INVALID;
    if (h->n == 0 || h->n >= 0x80000000u || h->m >= 0xFFFFFFFFu) return HGP_E_INVALID;
    if (!h->pin_off || !h->inc_off || !h->vwgt) return HGP_E_INVALID;
    if (h->m && !h->nwgt) return HGP_E_INVALID;
    if (h->p && (!h->pins || !h->inc)) return HGP_E_INVALID;
    return HGP_OK;
}

// Runs f, turning exceptions into status codes.  A call that fails after it
// has enqueued work (a workspace or capacity check partway through, a launch
// error) waits for `st` before returning, so that on every error return no
// work of the call is still running and the caller may reuse its buffers.
template <class F>
hgp_status guarded(hipStream_t st, F &&f) {
    hgp_status s;
    try {
        s = f();
    } catch (const Error &e) {
        s = e.code;
    } catch (...) {
        s = HGP_E_DEVICE;
    }
    if (s != HGP_OK) (void)hipStreamSynchronize(st);
    return s;
}

// Host-only computations (no stream involved).
template <class F>
hgp_status guarded_host(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        return e.code;
    } catch (...) {
        return HGP_E_DEVICE;
    }
}

size_t level_bytes(uint32_t n, uint32_t m, uint32_t p) {
    // arrays of one stored level: pin_off, pins, inc_off, inc, vwgt, nwgt, cid, part
    return 4ull * ((size_t)m + 1 + p + (size_t)n + 1 + p + n + m + n + n) + 8 * 256;
}

// Workspace of one lane: a bisection of an (n, m, p) hypergraph (its whole
// multilevel workspace, then the extraction of its sides in the same room).
size_t rb_lane_bytes(uint32_t n, uint32_t m, uint32_t p, const hgp_params &dp) {
    hgp_params p2 = dp;
    p2.k = 2;
    p2.ip = 0;
    p2.community = 0;
    size_t bis = 0;
    HGP_REQUIRE(hgp_workspace_bytes(HGP_OP_PARTITION, n, m, p, &p2, &bis) == HGP_OK, HGP_E_INVALID);
    return bis + 4096;
}

// One depth's sides with their parents' sizes: per node with (n_i, m_i, p_i)
// the result (n_i words) and per side pin_off, pins, inc_off, inc, vwgt, nwgt
// and two maps, 36 n_i + 16 m_i + 16 p_i + 16 bytes and 17 allocations.  Over
// a depth the n_i sum to at most n and the p_i to at most p; a side's nets
// each have a pin, so the m_i sum to at most max(m, p); at most k nodes.
size_t rb_region_bytes(uint32_t n, uint32_t m, uint32_t p, uint32_t k) {
    return 4ull * (9ull * n + 4ull * std::max(m, p) + 4ull * p + 4ull * k) + 17ull * 256 * k + 4096;
}

// The sides of every bisected node: a region per depth that bisects
// (ceil(log2 k) of them).
size_t rb_sides_bytes(uint32_t n, uint32_t m, uint32_t p, uint32_t k) {
    uint32_t depths = 1;
    while ((1u << depths) < k) ++depths;
    return (size_t)depths * rb_region_bytes(n, m, p, k);
}

// Recursive bipartitioning: the start map, the sides of every bisected node
// and one lane (more lanes run at once when the workspace holds them).
size_t rb_bytes(uint32_t n, uint32_t m, uint32_t p, const hgp_params &dp) {
    return 4ull * n + rb_sides_bytes(n, m, p, dp.k) + rb_lane_bytes(n, m, p, dp) + 8192;
}

}  // namespace

extern "C" {

hgp_status hgp_default_params(uint32_t k, hgp_params *out) {
    if (!out) return HGP_E_INVALID;
    out->k = k;
    out->eps_num = 3;
    out->eps_den = 100;
    out->seed = 0;
    out->limit_factor = 160;
    out->coarsen_subrounds = 3;
    out->lp_subrounds = 5;
    out->lp_rounds = 5;
    out->flags = 0;
    out->community = 0;
    out->ip = 0;
    return HGP_OK;
}

hgp_status hgp_workspace_bytes(int op, uint32_t n, uint32_t m, uint32_t p, const hgp_params *prm, size_t *out) {
    if (!out) return HGP_E_INVALID;
    hgp_params dp;
    uint32_t k = 2;
    if (prm) {
        hgp_status s = check_params(prm);
        if (s != HGP_OK) return s;
        dp = *prm;
        k = prm->k;
    } else {
        hgp_default_params(2, &dp);
    }
    return guarded_host([&]() -> hgp_status {
        size_t need = 0;
        switch (op) {
            case HGP_OP_COARSEN: need = coarsen_workspace(n, m, p, dp); break;
            case HGP_OP_CONTRACT: need = contract_workspace(n, m, p); break;
            case HGP_OP_REFINE: need = refine_workspace(n, m, k); break;
            case HGP_OP_VALIDATE: need = util_workspace(n, m); break;
            case HGP_OP_INITIAL: need = ip_workspace(n, m, p, k); break;
            case HGP_OP_GAINS: need = gaintable_workspace(n, m, k, n); break;  // also the graph tables
            case HGP_OP_COMMUNITY: need = community_workspace(n, m, p); break;
            case HGP_OP_PARTITION: {
                size_t temp = std::max({coarsen_workspace(n, m, p, dp), contract_workspace(n, m, p),
                                        refine_workspace(n, m, k), ip_workspace(n, m, p, k), util_workspace(n, m)});
                // hierarchy: every coarse level with the capacities of its
                // parent, and the maps, budgeted at eight input levels (the
                // input and levels whose sizes sum to at most seven times it
                // fit); on top, rep
                size_t hier = 8 * level_bytes(n, m, p) + 4ull * n + 4096;
                // community-aware coarsening: the detection runs first (its
                // scratch is free again before coarsening), and every level
                // keeps its vertices' communities
                if (dp.community) {
                    temp = std::max(temp, community_workspace(n, m, p));
                    hier += 8 * (4ull * n + 256) + 4ull * n;
                }
                need = temp + hier;
                if (dp.ip == 1) need += rb_bytes(n, m, p, dp);  // of the coarsest level (at most the input)
                break;
            }
            case HGP_OP_RB: need = rb_bytes(n, m, p, dp); break;
            default: return HGP_E_INVALID;
        }
        *out = need + 4096;
        return HGP_OK;
    });
}

hgp_status hgp_validate(const hgp_hg *h, void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (!ws) return HGP_E_WORKSPACE;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        return validate(*h, A, S(stream));
    });
}

hgp_status hgp_coarsen(const hgp_hg *h, const hgp_params *prm, uint32_t level, uint32_t *rep, uint32_t *n_clusters,
                       void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s == HGP_OK) s = check_params(prm);
    if (s != HGP_OK) return s;
    if (!rep || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        coarsen_pass(*h, *prm, level, rep, n_clusters, nullptr, A, S(stream));
        return HGP_OK;
    });
}

hgp_status hgp_contract(const hgp_hg *fine, const uint32_t *rep, uint32_t *cid, const hgp_hg_out *out, void *ws,
                        size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(fine);
    if (s != HGP_OK) return s;
    if (!rep || !cid || !out || !ws || !out->pin_off || !out->inc_off || !out->vwgt) return HGP_E_INVALID;
    if (out->cap_n < 1 || (fine->m && !out->nwgt) || (fine->p && (!out->pins || !out->inc))) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        contract(*fine, rep, cid, *out, nullptr, A, S(stream));
        return HGP_OK;
    });
}

hgp_status hgp_project(uint32_t n, const uint32_t *cid, const uint32_t *coarse_part, uint32_t *part, void *stream) {
    if (n && (!cid || !coarse_part || !part)) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        project(n, cid, coarse_part, part, S(stream));
        return HGP_OK;
    });
}

hgp_status hgp_objective(const hgp_hg *h, uint32_t k, const uint32_t *part, int64_t *objective, int64_t *block_wgt,
                         void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !objective || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        hgp::objective(*h, k, part, objective, block_wgt, A, S(stream));
        return HGP_OK;
    });
}

hgp_status hgp_refine_lp(const hgp_hg *h, const hgp_params *prm, uint32_t level, uint32_t *part, int64_t *objective,
                         int64_t *block_wgt, void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s == HGP_OK) s = check_params(prm);
    if (s != HGP_OK) return s;
    if (!part || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        refine_lp(*h, *prm, level, part, objective, block_wgt, A, S(stream));
        return HGP_OK;
    });
}

hgp_status hgp_initial_partition(const hgp_hg *h, uint32_t k, uint32_t *part, void *ws, size_t ws_bytes,
                                 void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        initial_partition(*h, k, part, A, S(stream));
        return HGP_OK;
    });
}

}  // extern "C"

namespace {
hgp_status rb_initial_partition(const hgp_hg &h, const hgp_params &prm, uint32_t *part, Arena &A, hipStream_t st);
}

extern "C" hgp_status hgp_rb_initial_partition(const hgp_hg *h, const hgp_params *prm, uint32_t *part, void *ws,
                                               size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s == HGP_OK) s = check_params(prm);
    if (s != HGP_OK) return s;
    if (!part || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        if (!(prm->flags & HGP_TRUSTED_INPUT)) {
            const hgp_status v = validate(*h, A, S(stream));
            if (v != HGP_OK) return v;
        }
        return rb_initial_partition(*h, *prm, part, A, S(stream));
    });
}

namespace {

// The multilevel driver (paper Alg. 1 with the deterministic components, no
// FM / flows) on one hypergraph, scratch from A, work on st.  Syncs.  Throws
// Error on workspace or device failures.  side_limits / fill_target: the
// block limits and the fill target of a bisection of the recursive
// bipartitioning (k = 2), or null / -1.
hgp_status partition_one(const hgp_hg *h0, const hgp_params *prm, uint32_t *part, int64_t *objective,
                         uint32_t *levels_out, Arena &A, hipStream_t st, hgp_trace *trace = nullptr,
                         const int64_t *side_limits = nullptr, int64_t fill_target = -1) {
    if (!(prm->flags & HGP_TRUSTED_INPUT)) {
        const hgp_status v = validate(*h0, A, st);
        if (v != HGP_OK) return v;
    }
    const int64_t W = total_weight(h0->vwgt, h0->n, A, st);  // c(V): the same on every level
    struct Level {
        hgp_hg h;
        uint32_t *cid;  // map to the next coarser level
    };
    std::vector<Level> L;
    L.push_back({*h0, nullptr});
    // community-aware coarsening (Sec. 4.3): the communities of the input,
    // carried to every coarse level by the contraction map
    uint32_t *comm = nullptr;
    if (prm->community) {
        comm = A.alloc<uint32_t>(h0->n);
        const hgp_status cs = communities(*h0, prm->seed, comm, nullptr, A, st);
        if (cs != HGP_OK) return cs;
    }
    const uint64_t limit = (uint64_t)prm->limit_factor * prm->k;
    for (;;) {
        hgp_hg cur = L.back().h;
        if (!((uint64_t)cur.n > limit)) break;
        size_t mk = A.mark();
        uint32_t *cid = A.alloc<uint32_t>(cur.n);
        // the would-be coarse level, with the capacities of this level
        hgp_hg_out out;
        out.cap_n = cur.n; out.cap_m = cur.m; out.cap_p = cur.p;
        out.pin_off = A.alloc<uint32_t>((size_t)cur.m + 1);
        out.pins = A.alloc<uint32_t>(cur.p);
        out.inc_off = A.alloc<uint32_t>((size_t)cur.n + 1);
        out.inc = A.alloc<uint32_t>(cur.p);
        out.vwgt = A.alloc<int32_t>(cur.n);
        out.nwgt = A.alloc<int32_t>(cur.m);
        out.dims = nullptr;
        uint32_t *ccomm = comm ? A.alloc<uint32_t>(cur.n) : nullptr;  // the coarse level's communities
        size_t mk_rep = A.mark();
        uint32_t *rep = A.alloc<uint32_t>(cur.n);
        uint32_t cnt = 0;
        coarsen_pass(cur, *prm, (uint32_t)(L.size() - 1), rep, nullptr, &cnt, A, st, W, comm);
        if ((uint64_t)100 * (cur.n - cnt) <= (uint64_t)cur.n) {
            A.release(mk);
            break;
        }
        uint32_t dims[3];
        contract(cur, rep, cid, out, dims, A, st);
        if (comm) {
            community_down(cur.n, cid, comm, ccomm, st);
            comm = ccomm;
        }
        A.release(mk_rep);
        // the coarse level keeps the arrays of its parent's capacities: only
        // their used prefix is read, and no copy is spent on compacting them
        hgp_hg nh;
        nh.n = dims[0]; nh.m = dims[1]; nh.p = dims[2];
        nh.pin_off = out.pin_off; nh.pins = out.pins; nh.inc_off = out.inc_off; nh.inc = out.inc;
        nh.vwgt = out.vwgt; nh.nwgt = out.nwgt;
        L.back().cid = cid;
        L.push_back({nh, nullptr});
        if (L.size() > 4096) break;
    }
    const uint32_t nl = (uint32_t)L.size() - 1;
    // initial partition and LP on the coarsest level
    hgp_hg cs = L.back().h;
    uint32_t *cpart = (nl == 0) ? part : A.alloc<uint32_t>(cs.n);
    // per-level record: sizes, and the LP rounds run (host, caller's arrays)
    auto rounds_of = [&](uint32_t l) -> uint32_t * {
        return (trace && trace->lp_rounds && l < trace->cap) ? trace->lp_rounds + l : nullptr;
    };
    if (prm->ip == 1) {
        const hgp_status rs = rb_initial_partition(cs, *prm, cpart, A, st);
        if (rs != HGP_OK) return rs;
    } else {
        initial_partition(cs, prm->k, cpart, A, st, W, fill_target);
    }
    refine_lp(cs, *prm, nl, cpart, objective, nullptr, A, st, W, rounds_of(nl), side_limits);
    for (int l = (int)nl - 1; l >= 0; --l) {
        hgp_hg fh = L[l].h;
        uint32_t *fpart = (l == 0) ? part : A.alloc<uint32_t>(fh.n);
        project(fh.n, L[l].cid, cpart, fpart, st);
        refine_lp(fh, *prm, (uint32_t)l, fpart, objective, nullptr, A, st, W, rounds_of((uint32_t)l), side_limits);
        cpart = fpart;
    }
    stream_sync(st);
    if (levels_out) *levels_out = nl;
    if (trace) {
        trace->levels = nl;
        for (uint32_t l = 0; l <= nl && l < trace->cap; ++l) {
            if (trace->n) trace->n[l] = L[l].h.n;
            if (trace->m) trace->m[l] = L[l].h.m;
            if (trace->p) trace->p[l] = L[l].h.p;
        }
    }
    return HGP_OK;
}

// Limits and fill targets of a bisection (Eq. 1): a subhypergraph of weight
// Wsub that gets kk of the ktot blocks of a hypergraph of weight Wtot; side 0
// takes ceil(kk/2) blocks.  eps' is computed in IEEE double with the C
// library's pow; side i's target is ceil(Wsub k_i / kk), its limit
// floor((1 + eps') target_i).
void rb_limits(int64_t Wtot, uint32_t ktot, const hgp_params &prm, int64_t Wsub, uint32_t kk, int64_t L[2],
               int64_t T[2]) {
    const uint32_t ks[2] = {(kk + 1) / 2, kk / 2};
    uint32_t lg = 0;
    while ((1u << lg) < kk) ++lg;
    const double eps = (double)prm.eps_num / (double)prm.eps_den;
    const double base = (1.0 + eps) * ((double)Wtot / (double)ktot) * ((double)kk / (double)Wsub);
    const double epsp = std::pow(base, 1.0 / (double)lg) - 1.0;
    for (int i = 0; i < 2; ++i) {
        T[i] = (Wsub * (int64_t)ks[i] + (int64_t)kk - 1) / (int64_t)kk;
        L[i] = (int64_t)std::floor((1.0 + epsp) * (double)T[i]);
    }
}

// The recursion runs depth by depth.  All bisections of one depth are
// independent (each writes only its own vertices' blocks and its own
// subhypergraphs), so up to RB_LANES of them run at once, each on a worker
// thread with its own stream and its own slice of the workspace; the results
// do not depend on how many run at once or in which order.
constexpr uint32_t RB_LANES = 8;

struct RbNode {  // a subhypergraph that gets kk blocks from b0 on
    hgp_hg H;
    uint32_t kk, b0;
    const uint32_t *vmap;  // its vertex i is vertex vmap[i] of the level being partitioned
};
struct RbSides {  // a bisected node: its result and both sides
    uint32_t *bp = nullptr;
    hgp_hg_out out[2];
    uint32_t *smap[2], *cmap[2];
    uint32_t dims[2][3];
};

// Bisects node nd (kk > 1, n > 0) and extracts both sides into o, or assigns
// its vertices to block b0 (kk == 1).  Work on ts, scratch from At; synced.
hgp_status rb_task(const hgp_params &prm, int64_t Wtot, uint32_t *part, const RbNode &nd, RbSides &o, Arena &At,
                   hipStream_t ts) {
    if (nd.kk == 1) {
        assign_block(nd.vmap, nd.H.n, nd.b0, part, ts);
        stream_sync(ts);
        return HGP_OK;
    }
    const size_t mk = At.mark();
    const int64_t Wsub = total_weight(nd.H.vwgt, nd.H.n, At, ts);
    int64_t L[2], T[2];
    rb_limits(Wtot, prm.k, prm, Wsub, nd.kk, L, T);
    int64_t *obj = At.alloc<int64_t>(1);
    hgp_params p2 = prm;
    p2.k = 2;
    p2.ip = 0;
    p2.community = 0;
    p2.flags |= HGP_TRUSTED_INPUT;  // built here, valid by construction
    const hgp_status s = partition_one(&nd.H, &p2, o.bp, obj, nullptr, At, ts, nullptr, L, T[0]);
    At.release(mk);
    if (s != HGP_OK) return s;
    for (uint32_t side = 0; side < 2; ++side) {
        subhypergraph(nd.H, o.bp, side, o.out[side], o.smap[side], o.dims[side], At, ts);
        gather_map(nd.vmap, o.smap[side], o.dims[side][0], o.cmap[side], ts);
    }
    stream_sync(ts);
    At.release(mk);
    return HGP_OK;
}

struct LaneStreams {  // created and destroyed with the recursion
    std::vector<hipStream_t> s;
    ~LaneStreams() {
        for (hipStream_t x : s) (void)hipStreamDestroy(x);
    }
};

// Bisected node's result and both sides, with the node's sizes as
// capacities, from the sides' arena.
void alloc_sides(Arena &R, const hgp_hg &H, RbSides &o) {
    o.bp = R.alloc<uint32_t>(H.n);
    for (int sd = 0; sd < 2; ++sd) {
        hgp_hg_out &out = o.out[sd];
        out.cap_n = H.n; out.cap_m = H.m; out.cap_p = H.p;
        out.pin_off = R.alloc<uint32_t>((size_t)H.m + 1);
        out.pins = R.alloc<uint32_t>(H.p);
        out.inc_off = R.alloc<uint32_t>((size_t)H.n + 1);
        out.inc = R.alloc<uint32_t>(H.p);
        out.vwgt = R.alloc<int32_t>(H.n);
        out.nwgt = R.alloc<int32_t>(H.m);
        out.dims = nullptr;
        o.smap[sd] = R.alloc<uint32_t>(H.n);
        o.cmap[sd] = R.alloc<uint32_t>(H.n);
    }
}

// Recursive bipartitioning (Sec. 5, Eq. 1): the k-way initial partition of h
// by bisections, each a multilevel cycle with k = 2 and the side limits of
// Eq. 1; side 0 of a node with kk blocks takes the first ceil(kk/2) of them.
// The nodes form a queue: a lane takes a node, bisects it and queues both
// sides, so a side is bisected as soon as its parent is done (not when the
// parent's whole depth is).  Each node writes only its own vertices' blocks
// and its own sides, so the results do not depend on the order.
hgp_status rb_initial_partition(const hgp_hg &h, const hgp_params &prm, uint32_t *part, Arena &A, hipStream_t st) {
    const size_t mk = A.mark();
    uint32_t *vmap = A.alloc<uint32_t>(h.n);
    iota_u32(vmap, h.n, st);
    const int64_t Wtot = total_weight(h.vwgt, h.n, A, st);
    stream_sync(st);  // the level and vmap are complete before the lanes read them
    // every bisected node's sides, kept to the end: the nodes of one depth
    // sum to at most one region, and ceil(log2 k) depths bisect
    const size_t sbytes = rb_sides_bytes(h.n, h.m, h.p, prm.k);
    Arena R(A.alloc<char>(sbytes), sbytes);
    // lanes: as many bisection workspaces of the largest node (the root) as
    // the workspace holds, at least one
    const size_t lb = rb_lane_bytes(h.n, h.m, h.p, prm);
    // (one lane while kernels are timed: the timing state is not shared)
    const size_t most = timing().mask ? 1 : RB_LANES;
    const uint32_t nl = (uint32_t)std::max<size_t>(1, std::min<size_t>(most, A.remaining() / lb));
    std::vector<Arena> lane;
    for (uint32_t i = 0; i < nl; ++i) lane.emplace_back(A.alloc<char>(lb), lb);
    int dev = 0;
    HGP_CHECK_HIP(hipGetDevice(&dev));
    LaneStreams ls;
    for (uint32_t i = 0; i < nl; ++i) {
        hipStream_t x;
        HGP_CHECK_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        ls.s.push_back(x);
    }
    std::mutex mu;
    std::condition_variable cv;
    std::deque<RbNode> q{RbNode{h, prm.k, 0, vmap}};
    uint32_t busy = 0;
    hgp_status result = HGP_OK;
    auto work = [&](uint32_t li) {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv.wait(lk, [&] { return !q.empty() || busy == 0 || result != HGP_OK; });
            if (result != HGP_OK || q.empty()) return;  // (q empty here means busy == 0: all done)
            const RbNode nd = q.front();
            q.pop_front();
            ++busy;
            RbSides o;
            hgp_status s = HGP_OK;
            try {
                if (nd.kk >= 2) alloc_sides(R, nd.H, o);
            } catch (const Error &e) {
                s = e.code;
            }
            lk.unlock();
            if (s == HGP_OK) {
                try {
                    s = rb_task(prm, Wtot, part, nd, o, lane[li], ls.s[li]);
                } catch (const Error &e) {
                    s = e.code;
                } catch (...) {
                    s = HGP_E_DEVICE;
                }
                if (s != HGP_OK) (void)hipStreamSynchronize(ls.s[li]);  // nothing of the failed task still runs
            }
            lk.lock();
            --busy;
            if (s != HGP_OK) {
                if (result == HGP_OK) result = s;
            } else if (nd.kk >= 2) {
                const uint32_t ks[2] = {(nd.kk + 1) / 2, nd.kk / 2};
                for (int sd = 0; sd < 2; ++sd) {
                    if (o.dims[sd][0] == 0) continue;  // an empty side gets no vertices
                    const hgp_hg_out &out = o.out[sd];
                    q.push_back(RbNode{hgp_hg{o.dims[sd][0], o.dims[sd][1], o.dims[sd][2], out.pin_off, out.pins,
                                              out.inc_off, out.inc, out.vwgt, out.nwgt},
                                       ks[sd], sd == 0 ? nd.b0 : nd.b0 + ks[0], o.cmap[sd]});
                }
            }
            cv.notify_all();
        }
    };
    if (nl == 1) {
        work(0);
    } else {
        const bool bw = blocking_waits;
        std::vector<std::thread> th;
        for (uint32_t li = 0; li < nl; ++li)
            th.emplace_back([&, li]() {
                (void)hipSetDevice(dev);
                blocking_waits = bw;
                work(li);
            });
        for (std::thread &t : th) t.join();
    }
    A.release(mk);
    return result;
}
}  // namespace

extern "C" {

hgp_status hgp_partition(const hgp_hg *h0, const hgp_params *prm, uint32_t *part, int64_t *objective,
                         uint32_t *levels_out, void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h0);
    if (s == HGP_OK) s = check_params(prm);
    if (s != HGP_OK) return s;
    if (!part || !objective || !ws) return HGP_E_INVALID;
    hipStream_t st = S(stream);
    return guarded(st, [&]() -> hgp_status {
        Arena A(ws, ws_bytes);
        return partition_one(h0, prm, part, objective, levels_out, A, st);
    });
}

hgp_status hgp_gain_table(const hgp_hg *h, uint32_t k, const uint32_t *part, int32_t *benefit, int32_t *penalty,
                          void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !benefit || !penalty || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        gain_table(*h, k, part, benefit, penalty, A, S(stream));
        return HGP_OK;
    });
}

hgp_status hgp_gain_table_update(const hgp_hg *h, uint32_t k, uint32_t *part, const uint32_t *node,
                                 const uint32_t *target, uint32_t count, int32_t *benefit, int32_t *penalty,
                                 void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !benefit || !penalty || !ws || (count && (!node || !target)) || count > h->n) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        return gain_table_update(*h, k, part, node, target, count, benefit, penalty, A, S(stream));
    });
}

hgp_status hgp_gain_recalc(const hgp_hg *h, uint32_t k, const uint32_t *part, const uint32_t *node,
                           const uint32_t *target, uint32_t count, int64_t *gain, void *ws, size_t ws_bytes,
                           void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !ws || (count && (!node || !target || !gain)) || count > h->n) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        return gain_recalc(*h, k, part, node, target, count, gain, A, S(stream));
    });
}

hgp_status hgp_communities(const hgp_hg *h, uint64_t seed, uint32_t *comm, uint32_t *levels_out, void *ws,
                           size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (!comm || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        return communities(*h, seed, comm, levels_out, A, S(stream));
    });
}

hgp_status hgp_graph_gain_table(const hgp_hg *h, uint32_t k, const uint32_t *part, int32_t *omega, void *ws,
                                size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !omega || !ws) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        return graph_gain_table(*h, k, part, omega, A, S(stream));
    });
}

hgp_status hgp_graph_moves(const hgp_hg *h, uint32_t k, uint32_t *part, const uint32_t *node, const uint32_t *target,
                           uint32_t count, int32_t *omega, int64_t *gain, void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h);
    if (s != HGP_OK) return s;
    if (k < 2) return HGP_E_INVALID;
    if (k > 256) return HGP_E_UNSUPPORTED;
    if (!part || !ws || (count && (!node || !target)) || count > h->n) return HGP_E_INVALID;
    return guarded(S(stream), [&]() {
        Arena A(ws, ws_bytes);
        return graph_moves(*h, k, part, node, target, count, omega, gain, A, S(stream));
    });
}

hgp_status hgp_partition_traced(const hgp_hg *h0, const hgp_params *prm, uint32_t *part, int64_t *objective,
                                hgp_trace *trace, void *ws, size_t ws_bytes, void *stream) {
    hgp_status s = check_hg(h0);
    if (s == HGP_OK) s = check_params(prm);
    if (s != HGP_OK) return s;
    if (!part || !objective || !ws || !trace) return HGP_E_INVALID;
    hipStream_t st = S(stream);
    return guarded(st, [&]() -> hgp_status {
        Arena A(ws, ws_bytes);
        return partition_one(h0, prm, part, objective, nullptr, A, st, trace);
    });
}

const char *hgp_status_str(hgp_status s) {
    switch (s) {
        case HGP_OK: return "ok";
        case HGP_E_INVALID: return "invalid argument or malformed input";
        case HGP_E_OVERFLOW: return "total weight would overflow 2^31";
        case HGP_E_WORKSPACE: return "workspace too small";
        case HGP_E_DEVICE: return "HIP runtime or launch error";
        case HGP_E_UNSUPPORTED: return "unsupported parameter (k > 256)";
        default: return "unknown status";
    }
}

}  // extern "C"
