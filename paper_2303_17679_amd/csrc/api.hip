// extern "C" entry points: argument checks, workspace arena, the multilevel
// driver (paper Alg. 1 with the deterministic components, no FM / flows).
#include "kernels.h"
#include <algorithm>
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
    if (p->community > 1) return HGP_E_INVALID;
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
            case HGP_OP_INITIAL: need = ip_workspace(n, p, k); break;
            case HGP_OP_GAINS: need = gaintable_workspace(n, m, k, n); break;  // also the graph tables
            case HGP_OP_COMMUNITY: need = community_workspace(n, m, p); break;
            case HGP_OP_PARTITION: {
                size_t temp = std::max({coarsen_workspace(n, m, p, dp), contract_workspace(n, m, p),
                                        refine_workspace(n, m, k), ip_workspace(n, p, k), util_workspace(n, m)});
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
                break;
            }
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
// The multilevel driver (paper Alg. 1 with the deterministic components, no
// FM / flows) on one hypergraph, scratch from A, work on st.  Syncs.  Throws
// Error on workspace or device failures.
hgp_status partition_one(const hgp_hg *h0, const hgp_params *prm, uint32_t *part, int64_t *objective,
                         uint32_t *levels_out, Arena &A, hipStream_t st, hgp_trace *trace = nullptr) {
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
    initial_partition(cs, prm->k, cpart, A, st, W);
    refine_lp(cs, *prm, nl, cpart, objective, nullptr, A, st, W, rounds_of(nl));
    for (int l = (int)nl - 1; l >= 0; --l) {
        hgp_hg fh = L[l].h;
        uint32_t *fpart = (l == 0) ? part : A.alloc<uint32_t>(fh.n);
        project(fh.n, L[l].cid, cpart, fpart, st);
        refine_lp(fh, *prm, (uint32_t)l, fpart, objective, nullptr, A, st, W, rounds_of((uint32_t)l));
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
