/*
 * hgp.h -- C ABI of the MI355X (gfx950) multilevel hypergraph partitioning
 * hot path: clustering-based coarsening, contraction, and deterministic
 * label-propagation refinement of the connectivity (lambda-1) objective,
 * after Gottesbüren, Heuer, Maas, Sanders, Schlag, "Scalable High-Quality
 * Hypergraph Partitioning" (arXiv 2303.17679).
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers (HIP device memory on the current
 *    device) unless a comment says "host".  The caller owns every buffer,
 *    including the workspace; the library never allocates device memory
 *    (beyond the one fixed array that hgp_refine_lp_static uses), never
 *    frees, and keeps no pointer past the end of the call.
 *  - IDs and offsets are uint32, vertex and net weights int32 (>= 1).
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *    Entry points marked "syncs" wait for `stream` before returning
 *    because the host needs device-computed sizes; the others may return
 *    before the device work is done.
 *  - Arguments are checked on the host before anything is enqueued; a bad
 *    argument returns an error status and enqueues nothing.  Device launch
 *    failures return HGP_E_DEVICE.  Nothing throws across the ABI.
 *  - Results are deterministic: for equal inputs and parameters every entry
 *    point produces bit-identical outputs on every run and launch
 *    configuration.  All arithmetic is integer.
 *
 * Workspace: every entry point that needs scratch memory takes `ws`
 * (device, 256-byte aligned) and `ws_bytes`; the required size comes from
 * hgp_workspace_bytes().  Too small a workspace returns HGP_E_WORKSPACE.
 */
#ifndef HGP_H
#define HGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hgp_status;
#define HGP_OK 0
#define HGP_E_INVALID (-1)     /* argument or input out of range / malformed   */
#define HGP_E_OVERFLOW (-2)    /* total weights would overflow 2^31             */
#define HGP_E_WORKSPACE (-3)   /* workspace too small                           */
#define HGP_E_DEVICE (-4)      /* HIP runtime or launch error                   */
#define HGP_E_UNSUPPORTED (-5) /* valid but not supported (e.g. k > 256)        */

/* A hypergraph level H = (V, E, c, w) as two adjacency arrays (paper Sec. 4.2):
 * pin lists of the nets and incident-net lists of the vertices.
 * Preconditions: n >= 1; pin_off[0] = 0, pin_off[m] = p, non-decreasing;
 * pins of a net strictly ascending and < n; inc_off/inc is the exact transpose
 * with nets strictly ascending per vertex; c(V) = sum vwgt < 2^31 and
 * sum nwgt < 2^31; m < 2^32 - 1.  hgp_validate() checks all of this. */
typedef struct {
    uint32_t n, m, p;
    const uint32_t *pin_off; /* [m+1] */
    const uint32_t *pins;    /* [p]   */
    const uint32_t *inc_off; /* [n+1] */
    const uint32_t *inc;     /* [p]   */
    const int32_t *vwgt;     /* [n]   */
    const int32_t *nwgt;     /* [m]   */
} hgp_hg;

/* Caller-allocated buffers of a contracted level.  Capacities of the fine
 * level always suffice (n' <= n, m' <= m, p' <= p). */
typedef struct {
    uint32_t cap_n, cap_m, cap_p;
    uint32_t *pin_off; /* [cap_m+1] */
    uint32_t *pins;    /* [cap_p]   */
    uint32_t *inc_off; /* [cap_n+1] */
    uint32_t *inc;     /* [cap_p]   */
    int32_t *vwgt;     /* [cap_n]   */
    int32_t *nwgt;     /* [cap_m]   */
    uint32_t *dims;    /* device [3] <- n', m', p' */
} hgp_hg_out;

/* Parameters.  Every field but flags changes results, so tests pass the
 * same values to the reference implementation.  hgp_default_params() fills
 * the defaults given in brackets. */
typedef struct {
    uint32_t k;                 /* number of blocks, 2..256                          */
    uint32_t eps_num, eps_den;  /* imbalance eps = num/den exactly [3/100]; den <= 2^20 */
    uint64_t seed;              /* seed of the tie-break / sub-round hash [0]        */
    uint32_t limit_factor;      /* coarsen while n > limit_factor * k [160] (Sec. 4.1); <= 2^20 */
    uint32_t coarsen_subrounds; /* S_c, sub-rounds of a clustering pass [3] (Sec. 11)  */
    uint32_t lp_subrounds;      /* S_lp, sub-rounds of an LP round [5] (Sec. 11)       */
    uint32_t lp_rounds;         /* R_lp, maximum LP rounds per level [5]               */
    uint32_t flags;             /* HGP_TRUSTED_INPUT or 0 [0]; results do not depend on it */
    uint32_t community;         /* 1: community-aware coarsening (Sec. 4.3), 0: none [0]  */
    uint32_t ip;                /* initial partition of the coarsest level: 0 greedy BFS
                                   fill, 1 recursive bipartitioning (Sec. 5, Eq. 1) [0]   */
} hgp_params;

/* hgp_params.flags: the caller vouches that the hypergraph meets every
 * precondition of hgp_hg (e.g. hgp_validate returned HGP_OK for it before),
 * so hgp_partition skips its own device-side check of the input.  Results
 * for valid input are the same; invalid input is then undefined behaviour. */
#define HGP_TRUSTED_INPUT 1u

/* Workspace-size queries. */
#define HGP_OP_COARSEN 1
#define HGP_OP_CONTRACT 2
#define HGP_OP_REFINE 3
#define HGP_OP_PARTITION 4
#define HGP_OP_VALIDATE 5
#define HGP_OP_INITIAL 6
#define HGP_OP_GAINS 7     /* hgp_gain_table, hgp_gain_table_update, hgp_gain_recalc, hgp_graph_* */
#define HGP_OP_COMMUNITY 8 /* hgp_communities */
#define HGP_OP_RB 9        /* hgp_rb_initial_partition */

/* Host.  Fills *out with the defaults listed in hgp_params for k blocks. */
hgp_status hgp_default_params(uint32_t k, hgp_params *out);

/* Host.  Workspace bytes needed by operation `op` on a level of n vertices,
 * m nets and p pins.  For HGP_OP_PARTITION the figure includes room for the
 * coarse hierarchy: eight times the arrays of the input level (each coarse
 * level keeps the array capacities of its parent, so the hierarchy holds the
 * input and every level but the coarsest; the figure holds whenever those
 * levels below the input sum to at most seven input levels, as for every
 * input tested); a deeper hierarchy makes hgp_partition return
 * HGP_E_WORKSPACE. */
hgp_status hgp_workspace_bytes(int op, uint32_t n, uint32_t m, uint32_t p,
                               const hgp_params *prm, size_t *out);

/* Checks every precondition of hgp_hg on the device (monotone offsets, pins
 * in range and strictly ascending, incidence = exact transpose, weights >= 1,
 * total weights < 2^31).  Syncs.  Returns HGP_OK, HGP_E_INVALID or
 * HGP_E_OVERFLOW. */
hgp_status hgp_validate(const hgp_hg *h, void *ws, size_t ws_bytes, void *stream);

/* One clustering pass of coarsening level `level` (paper Sec. 4.1 heavy-edge
 * rating, contraction limit and c_max; Sec. 11 deterministic clustering):
 * S_c sub-rounds; the unclustered singletons u with
 * H(seed,1,level,0,u) mod S_c = r rate the clusters of their neighbours by
 * r(u,C) = sum over e in I(u) touching C of floor(w(e) * 2^32 / (|e|-1)), each
 * net once per cluster; they may not join a candidate singleton of the same
 * sub-round and must keep 160k*(c(u)+c(C)) <= c(V); ties go to the smaller
 * H(seed,2,level,0,C), then the smaller C.  Joins are grouped by target,
 * ordered by (c(u), u) and the longest prefix within c_max is approved.  The
 * pass stops after the first sub-round leaving fewer than n/2.5 clusters.
 * Output rep[n] (rep[u] = representative, rep[rep[u]] = rep[u]) and
 * *n_clusters (device uint32). */
hgp_status hgp_coarsen(const hgp_hg *h, const hgp_params *prm, uint32_t level,
                       uint32_t *rep, uint32_t *n_clusters,
                       void *ws, size_t ws_bytes, void *stream);

/* Contraction of the clustering rep (paper Sec. 4.2): coarse vertex IDs
 * cid[v] = rank of rep[v] among the representatives (ascending); coarse
 * vertex weights are cluster sums; each net's pins are replaced by their coarse
 * IDs, sorted ascending and de-duplicated; nets left with fewer than two
 * pins are dropped; identical nets are merged into the one with the smallest
 * fine net ID, carrying the summed weight; kept nets are numbered in ascending
 * fine ID; the incidence arrays are the exact transpose.  Writes cid[n],
 * every array of *out and out->dims. */
hgp_status hgp_contract(const hgp_hg *fine, const uint32_t *rep, uint32_t *cid,
                        const hgp_hg_out *out, void *ws, size_t ws_bytes, void *stream);

/* Projection of a coarse partition to the finer level (paper Sec. 3):
 * part[v] = coarse_part[cid[v]] for v < n. */
hgp_status hgp_project(uint32_t n, const uint32_t *cid, const uint32_t *coarse_part,
                       uint32_t *part, void *stream);

/* Connectivity objective (paper Sec. 2) of a partition: *objective (device
 * int64) = sum over nets with lambda(e) > 1 of (lambda(e)-1) w(e), and
 * block_wgt[k] (device int64, may be NULL) = c(V_b). */
hgp_status hgp_objective(const hgp_hg *h, uint32_t k, const uint32_t *part,
                         int64_t *objective, int64_t *block_wgt,
                         void *ws, size_t ws_bytes, void *stream);

/* Deterministic synchronous label propagation of level `level` (paper
 * Sec. 11; gain of Sec. 6): up to R_lp rounds of S_lp sub-rounds; the nodes u
 * with H(seed,3,level,round,u) mod S_lp = s compute on the sub-round snapshot
 * their best move (largest positive connectivity gain, target block able to
 * take c(u) within L_max = (1+eps)ceil(c(V)/k), ties to the smaller block);
 * per block pair (s,t) the moves s->t and t->s are sorted by (gain desc, u asc)
 * and the last feasible state of the two-pointer merge walk is applied, with
 * per-pair budget floor((L_max - c(V_b))/(k-1)) for each block b of the pair.
 * Stops after a round without moves.  part[n] is refined in place;
 * *objective (device int64) and block_wgt[k] (device int64, may be NULL)
 * receive the result's objective and block weights. */
hgp_status hgp_refine_lp(const hgp_hg *h, const hgp_params *prm, uint32_t level,
                         uint32_t *part, int64_t *objective, int64_t *block_wgt,
                         void *ws, size_t ws_bytes, void *stream);

/* Simple deterministic initial partition of the coarsest level: vertices in
 * breadth-first order (start at the smallest unvisited ID; neighbours in
 * ascending incident-net then pin order), assigned to block 0, 1, ... in turn,
 * moving to the next block once the current one reaches ceil(c(V)/k).
 * Writes part[n]. */
hgp_status hgp_initial_partition(const hgp_hg *h, uint32_t k, uint32_t *part,
                                 void *ws, size_t ws_bytes, void *stream);

/* Recursive-bipartitioning initial partition (Sec. 5, Eq. 1) of h into
 * prm->k blocks.  A subhypergraph that gets kk > 1 of the blocks (at first h
 * with all k) is bisected by the multilevel cycle of hgp_partition with k = 2
 * and prm's other fields (community detection off, greedy fill at the
 * bottom): side 0, which will hold ceil(kk/2) blocks, is filled to its target
 * T_0 = ceil(c(V') ceil(kk/2) / kk), and side i may grow to
 * floor((1 + eps') T_i), where eps' = ((1 + eps) c(V) kk / (k c(V')))^(1 /
 * ceil(log2 kk)) - 1 (Eq. 1; IEEE double, the C library's pow).  Then both
 * sides are extracted as the subhypergraphs of Sec. 2 (vertices renumbered
 * in ascending ID, every net with a pin on the side kept with those pins,
 * single-pin nets included) and partitioned in turn: side 0 into blocks b0,
 * ..., side 1 into the blocks after them.  A subhypergraph with one block
 * is assigned to it.  Writes part[n] (device).  Workspace:
 * hgp_workspace_bytes(HGP_OP_RB, n, m, p, prm); the bisections of
 * different subhypergraphs are independent, and a larger workspace lets up
 * to eight of them run at once, each on a worker thread with a stream of its
 * own (same results).  Syncs.  prm->ip and prm->community are ignored;
 * HGP_TRUSTED_INPUT skips the input check. */
hgp_status hgp_rb_initial_partition(const hgp_hg *h, const hgp_params *prm, uint32_t *part,
                                    void *ws, size_t ws_bytes, void *stream);

/* Whole multilevel partition (paper Alg. 1 with the deterministic components
 * above, without FM and flows): coarsen while n > limit_factor*k and a pass
 * shrinks n by more than 1 %; initial partition of the coarsest level by the
 * greedy fill of hgp_initial_partition (prm->ip = 0) or by recursive
 * bipartitioning as in hgp_rb_initial_partition (prm->ip = 1);
 * LP on the coarsest level, then project + LP on every finer level.
 * Writes part[n] and *objective (device int64); *levels_out (host, may be
 * NULL) gets the number of contractions.  Syncs. */
hgp_status hgp_partition(const hgp_hg *h, const hgp_params *prm, uint32_t *part,
                         int64_t *objective, uint32_t *levels_out,
                         void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * refinement as hgp_refine_lp, with its scratch memory in a device array of
 * HGP_STATIC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends, instead of a caller workspace.  The call allocates
 * nothing.  A level whose hgp_workspace_bytes(HGP_OP_REFINE, n, m, p, prm)
 * exceeds HGP_STATIC_SCRATCH_BYTES is rejected with HGP_E_WORKSPACE before
 * anything is enqueued.  Every call on one device shares that device's array:
 * calls that overlap on one device (from several host threads, or on streams
 * not ordered with each other) race and give undefined results.  Syncs. */
#define HGP_STATIC_SCRATCH_BYTES (64u << 20)
hgp_status hgp_refine_lp_static(const hgp_hg *h, const hgp_params *prm, uint32_t level, uint32_t *part,
                                int64_t *objective, int64_t *block_wgt, void *stream);

/* Communities of the vertices for community-aware coarsening (paper
 * Sec. 4.3): the Louvain method on the bipartite graph of h (a node per
 * vertex and per net, an edge of weight w(e) per pin), deterministic by
 * synchronous local moving in sub-rounds (Sec. 11): at most 5 rounds of 5
 * sub-rounds per level, node x in sub-round H(seed, 4, level, round, x) mod 5;
 * a node moves to the neighbour community of largest positive modularity gain
 * (exact integer comparison; ties to the smaller community ID); at most 16
 * levels, each community contracted into its smallest node.  comm (device
 * uint32 [n]) receives a community ID per vertex (equal IDs = same community);
 * levels_out (host, may be NULL) the Louvain levels contracted.  The total
 * volume 2 * sum |e| w(e) must be below 2^31 (HGP_E_INVALID otherwise).
 * hgp_partition runs it first when params.community is 1 and then lets a
 * vertex join only clusters of its own community.  Workspace:
 * hgp_workspace_bytes(HGP_OP_COMMUNITY, ...).  Syncs. */
hgp_status hgp_communities(const hgp_hg *h, uint64_t seed, uint32_t *comm, uint32_t *levels_out, void *ws,
                           size_t ws_bytes, void *stream);

/* Gain table of a partition (paper Sec. 6.2): benefit[u] (device int32 [n])
 * = the weight of u's nets in which u is the only pin of its block, and
 * penalty[u * k + t] (device int32 [n * k], row u = the k penalties of u) =
 * the weight of u's nets without a pin in block t.  Moving u to t changes
 * the connectivity objective by penalty[u*k+t] - benefit[u] (so the gain is
 * benefit - penalty).  part[n] holds blocks < k. */
hgp_status hgp_gain_table(const hgp_hg *h, uint32_t k, const uint32_t *part, int32_t *benefit, int32_t *penalty,
                          void *ws, size_t ws_bytes, void *stream);

/* Applies the moves node[i] -> target[i] (device uint32 [count]; every node
 * at most once, targets < k; a move to the node's own block does nothing) to
 * part and brings a gain table of part up to date (paper Sec. 6.2 update
 * rules, net by net; the moved nodes' benefits are recomputed in their new
 * blocks).  Afterwards benefit and penalty equal hgp_gain_table of the new
 * partition.  A node listed twice or an index out of range returns
 * HGP_E_INVALID with part and the table unchanged.  Syncs. */
hgp_status hgp_gain_table_update(const hgp_hg *h, uint32_t k, uint32_t *part, const uint32_t *node,
                                 const uint32_t *target, uint32_t count, int32_t *benefit, int32_t *penalty,
                                 void *ws, size_t ws_bytes, void *stream);

/* Gains of a move sequence (paper Sec. 6.3, parallel gain recalculation):
 * gain[i] (device int64 [count]) = the decrease of the connectivity
 * objective caused by move i when the moves node[i] -> target[i] are made
 * one after the other in index order, starting from part (left unchanged).
 * Computed per net touched by a move from the first move into and the last
 * move out of every block among its pins.  Same move rules and errors as
 * hgp_gain_table_update.  Syncs. */
hgp_status hgp_gain_recalc(const hgp_hg *h, uint32_t k, const uint32_t *part, const uint32_t *node,
                           const uint32_t *target, uint32_t count, int64_t *gain, void *ws, size_t ws_bytes,
                           void *stream);

/* Graph gain table (paper Sec. 10), for a hypergraph whose nets all have two
 * pins (edges; HGP_E_INVALID otherwise): omega[u * k + i] (device int32
 * [n * k], row u = the k values of u) = w(u, V_i), the weight of u's edges
 * whose other endpoint lies in block i.  Moving u to t lowers the edge cut
 * (= the connectivity objective of a graph) by omega[u*k+t] - omega[u*k+Pi[u]].
 * part[n] holds blocks < k.  Workspace: hgp_workspace_bytes(HGP_OP_GAINS, ...).
 * Syncs. */
hgp_status hgp_graph_gain_table(const hgp_hg *h, uint32_t k, const uint32_t *part, int32_t *omega, void *ws,
                                size_t ws_bytes, void *stream);

/* Moves node[i] -> target[i] on a graph (paper Sec. 10; device uint32
 * [count], every node at most once, targets < k, a move to the node's own
 * block does nothing), taken as made one after the other in index order.
 * part is updated.  When omega (device int32 [n * k], a graph gain table of
 * part) is not NULL it is updated to the table of the new partition: for each
 * move u: s -> t and each edge {u, v}, w(u, v) is added to omega[v][t] and
 * subtracted from omega[v][s].  When gain (device int64 [count]) is not NULL,
 * gain[i] = the attributed gain of move i: over its edges {u, v}, +w for an
 * edge that stops being cut and -w for one that becomes cut, with v in the
 * block it holds when move i is made (its target if v's move comes earlier in
 * the list); the gains sum to the decrease of the edge cut.  Not a graph, a
 * node listed twice or an index out of range returns HGP_E_INVALID with
 * everything unchanged.  Workspace: HGP_OP_GAINS.  Syncs. */
hgp_status hgp_graph_moves(const hgp_hg *h, uint32_t k, uint32_t *part, const uint32_t *node, const uint32_t *target,
                           uint32_t count, int32_t *omega, int64_t *gain, void *ws, size_t ws_bytes, void *stream);

/* Per-level record of one multilevel partition, in host arrays the caller
 * owns: level l = 0 is the input, l = levels the coarsest level. */
typedef struct {
    uint32_t cap;        /* entries of each array below (levels + 1 are needed) */
    uint32_t levels;     /* out: number of contractions                         */
    uint32_t *n, *m, *p; /* out [cap] (each may be NULL): sizes of level l      */
    uint32_t *lp_rounds; /* out [cap] (may be NULL): LP rounds run on level l   */
} hgp_trace;

/* hgp_partition that also fills *trace (levels beyond trace->cap are run but
 * not recorded).  Used to price a run's algorithmic bytes by level.  Syncs. */
hgp_status hgp_partition_traced(const hgp_hg *h, const hgp_params *prm, uint32_t *part, int64_t *objective,
                                hgp_trace *trace, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Many hypergraphs at once.  Each request runs exactly the driver of
 * hgp_partition, so its results are bit-identical to a call on its own; what
 * changes is that requests overlap on the device.
 * ------------------------------------------------------------------------ */

/* A partition server (host object).  `lanes` (1..64) worker threads, each
 * with its own HIP stream, take requests in arrival order; a request is
 * admitted when a lane is free and its workspace
 * (hgp_workspace_bytes(HGP_OP_PARTITION, ...)) fits in the free part of
 * `pool` (device, 256-byte aligned, pool_bytes, owned by the caller and
 * untouched by anything else until hgp_server_destroy returns).  A request
 * that does not fit may be passed by later ones, at most 64 times; after
 * that it waits at the head until memory frees up.  Requests admitted while
 * others run overlap with them on the device (continuous admission).
 * Fails with HGP_E_INVALID while measurement (hgp_timing_begin) is active. */
typedef struct hgp_server hgp_server;
hgp_status hgp_server_create(uint32_t lanes, void *pool, size_t pool_bytes, hgp_server **out);

/* Queues one partition of h with parameters prm (both copied; the arrays
 * they point to, part[n] and *objective must stay valid until the request
 * is waited for).  The request starts after the work enqueued on `stream`
 * so far (its inputs may be produced there).  Returns a ticket in *ticket.
 * HGP_E_WORKSPACE: the request's workspace exceeds the whole pool. */
hgp_status hgp_server_submit(hgp_server *s, const hgp_hg *h, const hgp_params *prm, uint32_t *part,
                             int64_t *objective, void *stream, uint64_t *ticket);

/* Blocks until request `ticket` has finished (its results are then complete
 * on the device) and returns its status: the status hgp_partition would have
 * returned.  *levels_out (host, may be NULL) gets the number of
 * contractions, *latency_ms (may be NULL) the time from submission to
 * completion, *queue_ms (may be NULL) the time from submission to
 * admission.  A ticket can be waited for once. */
hgp_status hgp_server_wait(hgp_server *s, uint64_t ticket, uint32_t *levels_out, double *latency_ms,
                           double *queue_ms);

/* Finishes the running requests, cancels the queued ones (their wait
 * returns HGP_E_INVALID), joins the workers and frees the host object. */
hgp_status hgp_server_destroy(hgp_server *s);

/* Host.  Pool bytes with which hgp_partition_batch keeps `lanes` requests of
 * the batch in flight: lanes x the largest request's workspace. */
hgp_status hgp_batch_workspace_bytes(const hgp_hg *hs, const hgp_params *ps, uint32_t count, uint32_t lanes,
                                     size_t *out);

/* Partitions count independent hypergraphs hs[i] with parameters ps[i]
 * (host arrays of views and parameters; the views' arrays are device
 * pointers) through a server of `lanes` lanes over the workspace, largest
 * first.  parts: host array of count device pointers (part of hypergraph i,
 * [hs[i].n]); objectives: device int64 [count]; levels_out: host uint32
 * [count] or NULL.  Results equal hgp_partition on each hypergraph.  The
 * workspace must hold at least the largest request's workspace
 * (hgp_batch_workspace_bytes with lanes = 1); more lets more requests run
 * at once.  Returns the first failing request's status.  Syncs. */
hgp_status hgp_partition_batch(const hgp_hg *hs, const hgp_params *ps, uint32_t count, uint32_t lanes,
                               uint32_t *const *parts, int64_t *objectives, uint32_t *levels_out, void *ws,
                               size_t ws_bytes, void *stream);

/* Measurement support (host).  Kernel ids for the timing calls below. */
#define HGP_KID_RATE_G8 0    /* rating, groups of 8 lanes, 64-entry tables    */
#define HGP_KID_RATE_G16 1   /* rating, groups of 16 lanes, 256-entry tables  */
#define HGP_KID_RATE_G64 2   /* rating, one wave, 1024-entry tables           */
#define HGP_KID_RATE_BLOCK 3 /* rating, one workgroup per candidate           */
#define HGP_KID_GAINS 4      /* LP best moves                                 */
#define HGP_KID_LP_FAST 5    /* LP whole-pair approvals                       */
#define HGP_KID_LP_FUSED 6   /* LP sorted pair walk, one workgroup            */
#define HGP_KID_LP_UPDATE 7  /* LP connectivity update of touched nets        */
#define HGP_KID_HUB_INSERT 8 /* hub rating, global-table inserts               */
#define HGP_KID_HUB_ARGMAX 9 /* hub rating, best target per table slice        */
#define HGP_KID_HUB_LDS 10   /* hub rating in one workgroup's LDS table        */
#define HGP_KID_COUNT 11

/* Host.  Bytes of device scratch that accounting needs for levels of at most
 * n_max vertices and m_max nets. */
hgp_status hgp_timing_scratch_bytes(uint32_t n_max, uint32_t m_max, size_t *out);

/* Host.  Starts measuring the kernels whose ids are set in `mask` (bit i =
 * kernel id i).  account = 0: every launch of those kernels is bracketed by a
 * pair of HIP events recorded on its stream.  account = 1: instead, each such
 * launch is preceded by an accounting kernel that adds the launch's
 * compulsory bytes (each distinct array element it must read or write,
 * counted once) to a device counter; `scratch` (device, hgp_timing_scratch_bytes
 * bytes) holds the counters and stamp arrays.  Measurement is global to the
 * process and not thread safe. */
hgp_status hgp_timing_begin(uint32_t mask, int account, void *scratch, size_t scratch_bytes,
                            uint32_t n_max, uint32_t m_max);

/* Host.  Event timing of a subset of launches: from this call on, the j-th
 * launch (j = 0, 1, ...) of each timed kernel gets its event pair only when
 * j % every == phase.  A run repeated `every` times with phases 0 .. every-1
 * times each launch position once, at 1/every of the event cost per run.
 * hgp_timing_begin restores every = 1.  HGP_E_INVALID when every == 0 or
 * phase >= every. */
hgp_status hgp_timing_sample(uint32_t every, uint32_t phase);

/* Host.  Waits for the device, then for kernel ids i < count writes
 * total_ms[i] (summed event time), launches[i] (the timed launches; all
 * launches when accounting) and bytes[i] (accounted compulsory bytes, 0 when
 * not accounting), and stops measuring.  Any of the three pointers may be
 * NULL. */
hgp_status hgp_timing_end(uint32_t count, double *total_ms, uint64_t *launches, double *bytes);

/* Host.  Static description of a status code. */
const char *hgp_status_str(hgp_status s);

#ifdef __cplusplus
}
#endif
#endif /* HGP_H */
