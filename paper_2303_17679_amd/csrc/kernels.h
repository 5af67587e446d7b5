// Host-side entry points of the translation units (internal).
#pragma once
#include "common.h"
#include <vector>

namespace hgp {

// util.hip
int64_t total_weight(const int32_t *w, uint32_t n, Arena &A, hipStream_t st);
int32_t max_vertex_weight(const int32_t *w, uint32_t n, Arena &A, hipStream_t st);
size_t util_workspace(uint32_t n, uint32_t m);
hgp_status validate(const hgp_hg &h, Arena &A, hipStream_t st);

// coarsen.hip
size_t coarsen_workspace(uint32_t n, uint32_t m, uint32_t p, const hgp_params &prm);
// W_known: c(V) when the caller knows it (it is the same on every level), or
// -1 to compute it here (one reduction and a sync).
// comm (device, may be null): community of every vertex; u joins only
// clusters of its own community (Sec. 4.3).
void coarsen_pass(const hgp_hg &h, const hgp_params &prm, uint32_t level, uint32_t *rep, uint32_t *n_clusters_dev,
                  uint32_t *n_clusters_host, Arena &A, hipStream_t st, int64_t W_known = -1,
                  const uint32_t *comm = nullptr);

// contract.hip
size_t contract_workspace(uint32_t n, uint32_t m, uint32_t p);
void contract(const hgp_hg &h, const uint32_t *rep, uint32_t *cid, const hgp_hg_out &out, uint32_t *dims_host,
              Arena &A, hipStream_t st);

// refine.hip
size_t refine_workspace(uint32_t n, uint32_t m, uint32_t k);
void objective(const hgp_hg &h, uint32_t k, const uint32_t *part, int64_t *obj, int64_t *bw, Arena &A,
               hipStream_t st);
// rounds_out (host, may be null): LP rounds run on the level.  side_limits
// (host, may be null; k must be 2): the weight limits of blocks 0 and 1 of a
// bisection of the recursive bipartitioning, in place of L_max.
void refine_lp(const hgp_hg &h, const hgp_params &prm, uint32_t level, uint32_t *part, int64_t *obj, int64_t *bw,
               Arena &A, hipStream_t st, int64_t W_known = -1, uint32_t *rounds_out = nullptr,
               const int64_t *side_limits = nullptr);

// ip.hip
size_t ip_workspace(uint32_t n, uint32_t m, uint32_t p, uint32_t k);
// fill_target >= 0: every block is filled to it instead of ceil(c(V)/k) (a
// bisection fills block 0 to its share; the last block takes the rest).
void initial_partition(const hgp_hg &h, uint32_t k, uint32_t *part, Arena &A, hipStream_t st, int64_t W_known = -1,
                       int64_t fill_target = -1);
void project(uint32_t n, const uint32_t *cid, const uint32_t *cpart, uint32_t *part, hipStream_t st);

// community.hip
size_t community_workspace(uint32_t n, uint32_t m, uint32_t p);
hgp_status communities(const hgp_hg &h, uint64_t seed, uint32_t *comm, uint32_t *levels_out, Arena &A,
                       hipStream_t st);
// ccomm[cid[u]] = comm[u] for u < n: the communities of a contracted level
void community_down(uint32_t n, const uint32_t *cid, const uint32_t *comm, uint32_t *ccomm, hipStream_t st);

// rb.hip: the subhypergraph of the vertices with part[v] == side (Sec. 2
// definition) into out (capacities of h suffice); vmap[i] <- the vertex of h
// that vertex i of the subhypergraph stands for; dims_host <- n', m', p'.
// Syncs.
void subhypergraph(const hgp_hg &h, const uint32_t *part, uint32_t side, const hgp_hg_out &out, uint32_t *vmap,
                   uint32_t *dims_host, Arena &A, hipStream_t st);
void gather_map(const uint32_t *outer, const uint32_t *inner, uint32_t n, uint32_t *out, hipStream_t st);
void assign_block(const uint32_t *vmap, uint32_t n, uint32_t b, uint32_t *part, hipStream_t st);
void iota_u32(uint32_t *p, uint32_t n, hipStream_t st);

// gaintable.hip
size_t gaintable_workspace(uint32_t n, uint32_t m, uint32_t k, uint32_t count);
void gain_table(const hgp_hg &h, uint32_t k, const uint32_t *part, int32_t *ben, int32_t *pen, Arena &A,
                hipStream_t st);
hgp_status gain_table_update(const hgp_hg &h, uint32_t k, uint32_t *part, const uint32_t *node,
                             const uint32_t *target, uint32_t count, int32_t *ben, int32_t *pen, Arena &A,
                             hipStream_t st);
hgp_status gain_recalc(const hgp_hg &h, uint32_t k, const uint32_t *part, const uint32_t *node,
                       const uint32_t *target, uint32_t count, int64_t *gain, Arena &A, hipStream_t st);
// graphs (every net two pins): w(u, V_i) table and moves with attributed gains
hgp_status graph_gain_table(const hgp_hg &h, uint32_t k, const uint32_t *part, int32_t *omega, Arena &A,
                            hipStream_t st);
hgp_status graph_moves(const hgp_hg &h, uint32_t k, uint32_t *part, const uint32_t *node, const uint32_t *target,
                       uint32_t count, int32_t *omega, int64_t *gain, Arena &A, hipStream_t st);

}  // namespace hgp
