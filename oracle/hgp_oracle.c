/*
 * hgp_oracle.c -- plain sequential CPU oracle of the multilevel hot path of
 * "Scalable High-Quality Hypergraph Partitioning" (Gottesbüren, Heuer, Maas,
 * Sanders, Schlag; arXiv 2303.17679).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is compared against.  Only the test suite,
 * the smoke check and the CPU baseline of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.
 *
 * Everything is integer arithmetic.  Each function names the part of the
 * paper it follows; where the paper is silent or ambiguous, the reading
 * taken is named R1..R14 (listed in the design notes of the repository).
 *
 * Pinning: every exported function is checked by the CPU test suite against
 * brute force from the definitions (objective, gains, ratings, contraction by
 * sets, pair selection by enumeration of the merge walk), closed-form special
 * cases and hand-derived golden fixtures.  The SplitMix64 finalizer used as
 * the seeded tie-break hash is pinned by published SplitMix64 output values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    uint32_t n, m, p;
    const uint32_t *pin_off, *pins;   /* nets -> pins, pins ascending per net   */
    const uint32_t *inc_off, *inc;    /* vertices -> nets, nets ascending        */
    const int32_t *vwgt, *nwgt;       /* c(v) >= 1, omega(e) >= 1                */
} or_hg;

typedef struct {
    uint32_t k;
    uint32_t eps_num, eps_den;        /* epsilon = eps_num / eps_den (R13)      */
    uint64_t seed;
    uint32_t limit_factor;            /* contraction limit 160 k (Sec. 4.1)    */
    uint32_t coarsen_subrounds;       /* S_c                                   */
    uint32_t lp_subrounds;            /* S_lp                                  */
    uint32_t lp_rounds;               /* R_lp                                  */
    uint32_t community;               /* 1: community-aware coarsening (4.3)   */
    uint32_t ip;                      /* 0: greedy BFS fill, 1: recursive      */
                                      /*    bipartitioning (Sec. 5, R19)       */
} or_params;

#define OR_NONE 0xFFFFFFFFu

enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_NOMEM = -3 };

/* ------------------------------------------------------------------------ */
/* Seeded hash (R5): the SplitMix64 finalizer applied to a tagged counter.   */
/* ------------------------------------------------------------------------ */
uint64_t or_mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

/* purpose: 1 coarsening sub-round, 2 rating tie, 3 LP sub-round. */
uint64_t or_hash(uint64_t seed, uint32_t purpose, uint32_t level, uint32_t it, uint32_t x)
{
    uint64_t tag = (uint64_t)((purpose & 0xFFu) | ((level & 0xFFu) << 8) | ((it & 0xFFFFu) << 16));
    return or_mix64(or_mix64(seed) ^ ((tag << 32) | (uint64_t)x));
}

/* ------------------------------------------------------------------------ */
/* Totals and the balance bound (Sec. 2, balanced partitioning problem).     */
/* ------------------------------------------------------------------------ */
int64_t or_total_weight(const or_hg *h)
{
    int64_t w = 0;
    for (uint32_t v = 0; v < h->n; ++v) w += h->vwgt[v];
    return w;
}

/* L_max = (1 + eps) * ceil(c(V) / k); an integer block weight c satisfies
 * c <= (1+eps)*ceil(W/k) exactly when c <= floor((den+num)*ceil(W/k)/den). */
int64_t or_lmax(int64_t W, uint32_t k, uint32_t eps_num, uint32_t eps_den)
{
    int64_t per = (W + (int64_t)k - 1) / (int64_t)k;
    return ((int64_t)(eps_den + eps_num) * per) / (int64_t)eps_den;
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

/* ------------------------------------------------------------------------ */
/* Connectivity objective (Sec. 2): f = sum over cut nets of (lambda-1)*w.   */
/* ------------------------------------------------------------------------ */
int64_t or_objective(const or_hg *h, uint32_t k, const uint32_t *part, int64_t *block_w)
{
    uint32_t *mark = (uint32_t *)malloc(sizeof(uint32_t) * (k ? k : 1));
    for (uint32_t b = 0; b < k; ++b) mark[b] = OR_NONE;
    int64_t f = 0;
    for (uint32_t e = 0; e < h->m; ++e) {
        uint32_t lambda = 0;
        for (uint32_t j = h->pin_off[e]; j < h->pin_off[e + 1]; ++j) {
            uint32_t b = part[h->pins[j]];
            if (mark[b] != e) { mark[b] = e; ++lambda; }
        }
        if (lambda > 1) f += (int64_t)(lambda - 1) * h->nwgt[e];
    }
    if (block_w) {
        for (uint32_t b = 0; b < k; ++b) block_w[b] = 0;
        for (uint32_t v = 0; v < h->n; ++v) block_w[part[v]] += h->vwgt[v];
    }
    free(mark);
    return f;
}

/* Pin count Phi(e, b) = |e intersect V_b| (Sec. 2). */
static uint32_t phi(const or_hg *h, const uint32_t *part, uint32_t e, uint32_t b)
{
    uint32_t c = 0;
    for (uint32_t j = h->pin_off[e]; j < h->pin_off[e + 1]; ++j)
        if (part[h->pins[j]] == b) ++c;
    return c;
}

/* Connectivity gain of moving u to block t (Sec. 6):
 * g = w({e in I(u): Phi(e, Pi[u]) = 1}) - w({e in I(u): Phi(e, t) = 0}). */
int64_t or_gain(const or_hg *h, const uint32_t *part, uint32_t u, uint32_t t)
{
    int64_t g = 0;
    uint32_t s = part[u];
    for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
        uint32_t e = h->inc[j];
        if (phi(h, part, e, s) == 1) g += h->nwgt[e];
        if (phi(h, part, e, t) == 0) g -= h->nwgt[e];
    }
    return g;
}

/* ------------------------------------------------------------------------ */
/* Coarsening: one clustering pass (Sec. 4.1 rating function and contraction */
/* limits; Sec. 11 deterministic clustering for coarsening).                 */
/* ------------------------------------------------------------------------ */

/* Heavy-edge rating score of one net, fixed point: floor(w(e) * 2^32 / (|e|-1)) (R14). */
static uint64_t net_score(int32_t w, uint32_t size)
{
    return (((uint64_t)(uint32_t)w) << 32) / (uint64_t)(size - 1);
}

/* Best target cluster of every candidate of sub-round r.  Candidates are the
 * unclustered singletons u with H(seed,1,level,0,u) mod S_c = r (Sec. 11).
 * rep/cw/csize are the snapshot at the start of the sub-round.  target[u] is
 * set for candidates (OR_NONE when no valid cluster exists) and left OR_NONE
 * for non-candidates.  Returns the number of candidates. */
static uint32_t rate_subround(const or_hg *h, const or_params *P, uint32_t level, uint32_t r,
                              const uint32_t *rep, const int64_t *cw, const uint32_t *csize,
                              const uint32_t *comm, uint32_t *target)
{
    const uint32_t n = h->n;
    const int64_t W = or_total_weight(h);
    const int64_t cap_mult = (int64_t)P->limit_factor * (int64_t)P->k; /* 160 k */
    uint8_t *cand = (uint8_t *)calloc(n ? n : 1, 1);
    uint64_t *R = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    uint64_t *seen = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    uint32_t *touched = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t stamp = 0;
    uint32_t ncand = 0;

    for (uint32_t u = 0; u < n; ++u) {
        target[u] = OR_NONE;
        cand[u] = (rep[u] == u && csize[u] == 1 &&
                   or_hash(P->seed, 1, level, 0, u) % P->coarsen_subrounds == r);
    }
    for (uint32_t u = 0; u < n; ++u) {
        if (!cand[u]) continue;
        ++ncand;
        uint32_t nt = 0;
        /* r(u, C) = sum over nets e in I(u) that also touch C of w(e)/(|e|-1);
         * each net counts once per cluster (R1). */
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            uint32_t e = h->inc[j];
            uint32_t size = h->pin_off[e + 1] - h->pin_off[e];
            if (size < 2) continue;
            uint64_t s = net_score(h->nwgt[e], size);
            ++stamp; /* one stamp per (candidate, net): de-duplicates clusters inside e */
            for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) {
                uint32_t v = h->pins[q];
                if (v == u) continue;
                uint32_t C = rep[v];
                if (seen[C] == stamp) continue;
                seen[C] = stamp;
                if (R[C] == 0) touched[nt++] = C; /* every score is >= 1 */
                R[C] += s;
            }
        }
        /* argmax over valid clusters; ties -> smaller H(seed,2,level,0,C) -> smaller C (R5). */
        uint32_t best = OR_NONE;
        uint64_t bestR = 0, bestH = 0;
        for (uint32_t q = 0; q < nt; ++q) {
            uint32_t C = touched[q];
            uint64_t rc = R[C];
            int valid = (C != rep[u]) &&
                        (cap_mult * ((int64_t)h->vwgt[u] + cw[C]) <= W) && /* R4 */
                        !cand[C] &&                                        /* R3 */
                        (!comm || comm[C] == comm[u]);                     /* Sec. 4.3 */
            if (valid) {
                uint64_t hc = or_hash(P->seed, 2, level, 0, C);
                if (best == OR_NONE || rc > bestR ||
                    (rc == bestR && (hc < bestH || (hc == bestH && C < best)))) {
                    best = C; bestR = rc; bestH = hc;
                }
            }
        }
        for (uint32_t q = 0; q < nt; ++q) { R[touched[q]] = 0; }
        target[u] = best;
    }
    free(cand); free(R); free(seen); free(touched);
    return ncand;
}

uint32_t or_rate_subround(const or_hg *h, const or_params *P, uint32_t level, uint32_t r,
                          const uint32_t *rep, const int64_t *cw, const uint32_t *csize,
                          uint32_t *target)
{
    return rate_subround(h, P, level, r, rep, cw, csize, NULL, target);
}

/* The same with the community restriction of Sec. 4.3: u may join only a
 * cluster whose representative lies in u's community (comm[v] for every
 * vertex of the level). */
uint32_t or_rate_subround_c(const or_hg *h, const or_params *P, uint32_t level, uint32_t r,
                            const uint32_t *rep, const int64_t *cw, const uint32_t *csize,
                            const uint32_t *comm, uint32_t *target)
{
    return rate_subround(h, P, level, r, rep, cw, csize, comm, target);
}

typedef struct { uint32_t C; int32_t c; uint32_t u; } or_join;

static int cmp_join(const void *a, const void *b)
{
    const or_join *x = (const or_join *)a, *y = (const or_join *)b;
    if (x->C != y->C) return x->C < y->C ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    if (x->u != y->u) return x->u < y->u ? -1 : 1;
    return 0;
}

/* Approval (Sec. 11): group the moves by target cluster, order each group by
 * ascending node weight with the node ID as tie breaker, and apply the longest
 * prefix whose weight keeps the cluster within c_max (Sec. 4.1:
 * c_max = c(V)/(160k), tested exactly as 160k * c(C) <= c(V)).
 * Updates rep, cw, csize in place; returns the number of approved joins. */
uint32_t or_approve_apply(const or_hg *h, const or_params *P, const uint32_t *target,
                          uint32_t *rep, int64_t *cw, uint32_t *csize)
{
    const uint32_t n = h->n;
    const int64_t W = or_total_weight(h);
    const int64_t cap_mult = (int64_t)P->limit_factor * (int64_t)P->k;
    uint32_t nj = 0;
    for (uint32_t u = 0; u < n; ++u) if (target[u] != OR_NONE) ++nj;
    or_join *J = (or_join *)malloc(sizeof(or_join) * (nj ? nj : 1));
    nj = 0;
    for (uint32_t u = 0; u < n; ++u)
        if (target[u] != OR_NONE) { J[nj].C = target[u]; J[nj].c = h->vwgt[u]; J[nj].u = u; ++nj; }
    qsort(J, nj, sizeof(or_join), cmp_join);
    /* decide on the snapshot cw, then apply */
    uint8_t *ok = (uint8_t *)calloc(nj ? nj : 1, 1);
    uint32_t i = 0, approved = 0;
    while (i < nj) {
        uint32_t C = J[i].C, g = i;
        int64_t prefix = 0;
        int open = 1;
        for (; g < nj && J[g].C == C; ++g) {
            prefix += J[g].c;
            if (open && cap_mult * (cw[C] + prefix) <= W) ok[g] = 1;
            else open = 0;
        }
        i = g;
    }
    for (uint32_t q = 0; q < nj; ++q) {
        if (!ok[q]) continue;
        rep[J[q].u] = J[q].C;
        cw[J[q].C] += J[q].c;
        csize[J[q].C] += 1;
        ++approved;
    }
    free(J); free(ok);
    return approved;
}

/* One clustering pass of level `level` (Sec. 4.1, Sec. 11).  rep is output.
 * The pass ends early after a sub-round in which the number of clusters drops
 * below n/2.5 of the current level (R2). */
static int cluster_pass(const or_hg *h, const or_params *P, uint32_t level, const uint32_t *comm,
                        uint32_t *rep, uint32_t *n_clusters, uint32_t *subrounds_run)
{
    const uint32_t n = h->n;
    int64_t *cw = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    uint32_t *csize = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *target = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!cw || !csize || !target) return OR_E_NOMEM;
    for (uint32_t u = 0; u < n; ++u) { rep[u] = u; cw[u] = h->vwgt[u]; csize[u] = 1; }
    uint32_t cnt = n, run = 0;
    for (uint32_t r = 0; r < P->coarsen_subrounds; ++r) {
        rate_subround(h, P, level, r, rep, cw, csize, comm, target);
        cnt -= or_approve_apply(h, P, target, rep, cw, csize);
        ++run;
        if ((uint64_t)5 * cnt < (uint64_t)2 * n) break;
    }
    *n_clusters = cnt;
    if (subrounds_run) *subrounds_run = run;
    free(cw); free(csize); free(target);
    return OR_OK;
}

int or_cluster_pass(const or_hg *h, const or_params *P, uint32_t level,
                    uint32_t *rep, uint32_t *n_clusters, uint32_t *subrounds_run)
{
    return cluster_pass(h, P, level, NULL, rep, n_clusters, subrounds_run);
}

/* A clustering pass restricted to communities (Sec. 4.3); comm[v] for every
 * vertex of the level. */
int or_cluster_pass_c(const or_hg *h, const or_params *P, uint32_t level, const uint32_t *comm,
                      uint32_t *rep, uint32_t *n_clusters, uint32_t *subrounds_run)
{
    return cluster_pass(h, P, level, comm, rep, n_clusters, subrounds_run);
}

/* ------------------------------------------------------------------------ */
/* Contraction (Sec. 4.2).                                                   */
/* ------------------------------------------------------------------------ */
static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct { uint64_t f; uint32_t size; uint32_t e; } or_fp;

static int cmp_fp(const void *a, const void *b)
{
    const or_fp *x = (const or_fp *)a, *y = (const or_fp *)b;
    if (x->f != y->f) return x->f < y->f ? -1 : 1;
    if (x->size != y->size) return x->size < y->size ? -1 : 1;
    if (x->e != y->e) return x->e < y->e ? -1 : 1;
    return 0;
}

/* Contract the clustering rep.  Output buffers are sized by the fine level:
 * c_pin_off[m+1], c_pins[p], c_inc_off[n+1], c_inc[p], c_vwgt[n], c_nwgt[m].
 * dims[0..2] <- n', m', p'.  cid[n] <- coarse vertex of every fine vertex. */
int or_contract(const or_hg *h, const uint32_t *rep, uint32_t *cid, uint32_t *dims,
                uint32_t *c_pin_off, uint32_t *c_pins, uint32_t *c_inc_off, uint32_t *c_inc,
                int32_t *c_vwgt, int32_t *c_nwgt)
{
    const uint32_t n = h->n, m = h->m;
    /* Remap node IDs to a consecutive range: representatives in ascending ID. */
    uint32_t *rank = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t nc = 0;
    for (uint32_t v = 0; v < n; ++v) { rank[v] = nc; if (rep[v] == v) ++nc; }
    for (uint32_t v = 0; v < n; ++v) cid[v] = rank[rep[v]];
    /* Supernode weight = sum of the weights of its cluster. */
    for (uint32_t c = 0; c < nc; ++c) c_vwgt[c] = 0;
    for (uint32_t v = 0; v < n; ++v) c_vwgt[cid[v]] += h->vwgt[v];

    /* Replace pins by their supernodes and discard repeated supernodes. */
    uint32_t *t_off = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *t_pins = (uint32_t *)malloc(sizeof(uint32_t) * (h->p ? h->p : 1));
    t_off[0] = 0;
    uint32_t w = 0;
    for (uint32_t e = 0; e < m; ++e) {
        uint32_t b = w;
        for (uint32_t j = h->pin_off[e]; j < h->pin_off[e + 1]; ++j) t_pins[w++] = cid[h->pins[j]];
        qsort(t_pins + b, w - b, sizeof(uint32_t), cmp_u32);
        uint32_t u = b;
        for (uint32_t j = b; j < w; ++j)
            if (j == b || t_pins[j] != t_pins[u - 1]) t_pins[u++] = t_pins[j];
        w = u;
        t_off[e + 1] = w;
    }

    /* Identical nets: fingerprints f(e) = sum of v^2 (mod 2^64), sort by
     * (fingerprint, size), compare pairwise inside runs; single-pin nets are
     * removed (they never contribute to the objective). */
    or_fp *F = (or_fp *)malloc(sizeof(or_fp) * (m ? m : 1));
    uint32_t nf = 0;
    for (uint32_t e = 0; e < m; ++e) {
        uint32_t size = t_off[e + 1] - t_off[e];
        if (size < 2) continue;
        uint64_t f = 0;
        for (uint32_t j = t_off[e]; j < t_off[e + 1]; ++j) f += (uint64_t)t_pins[j] * (uint64_t)t_pins[j];
        F[nf].f = f; F[nf].size = size; F[nf].e = e; ++nf;
    }
    qsort(F, nf, sizeof(or_fp), cmp_fp);
    uint32_t *rep_net = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    for (uint32_t e = 0; e < m; ++e) rep_net[e] = OR_NONE;
    uint32_t i = 0;
    while (i < nf) {
        uint32_t g = i;
        while (g < nf && F[g].f == F[i].f && F[g].size == F[i].size) ++g;
        for (uint32_t a = i; a < g; ++a) {
            uint32_t ea = F[a].e;
            rep_net[ea] = ea;
            for (uint32_t b = i; b < a; ++b) {
                uint32_t eb = F[b].e;
                if (rep_net[eb] != eb) continue;
                if (memcmp(t_pins + t_off[ea], t_pins + t_off[eb], sizeof(uint32_t) * F[a].size) == 0) {
                    rep_net[ea] = eb; /* run is in ascending net ID: eb is the smallest */
                    break;
                }
            }
        }
        i = g;
    }
    /* The kept net of each identical group carries the group's total weight. */
    int64_t *wsum = (int64_t *)calloc(m ? m : 1, sizeof(int64_t));
    for (uint32_t e = 0; e < m; ++e) if (rep_net[e] != OR_NONE) wsum[rep_net[e]] += h->nwgt[e];

    /* Kept nets are renumbered in ascending fine ID (prefix sum over the
     * validity bitset). */
    uint32_t mc = 0, pc = 0;
    c_pin_off[0] = 0;
    for (uint32_t e = 0; e < m; ++e) {
        if (rep_net[e] != e) continue;
        for (uint32_t j = t_off[e]; j < t_off[e + 1]; ++j) c_pins[pc++] = t_pins[j];
        c_nwgt[mc] = (int32_t)wsum[e];
        ++mc;
        c_pin_off[mc] = pc;
    }
    /* Incident nets: transpose of the pin lists, ascending net ID. */
    for (uint32_t v = 0; v <= nc; ++v) c_inc_off[v] = 0;
    for (uint32_t j = 0; j < pc; ++j) c_inc_off[c_pins[j] + 1]++;
    for (uint32_t v = 0; v < nc; ++v) c_inc_off[v + 1] += c_inc_off[v];
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (nc ? nc : 1));
    for (uint32_t v = 0; v < nc; ++v) cur[v] = c_inc_off[v];
    for (uint32_t e = 0; e < mc; ++e)
        for (uint32_t j = c_pin_off[e]; j < c_pin_off[e + 1]; ++j) c_inc[cur[c_pins[j]]++] = e;

    dims[0] = nc; dims[1] = mc; dims[2] = pc;
    free(rank); free(t_off); free(t_pins); free(F); free(rep_net); free(wsum); free(cur);
    return OR_OK;
}

/* Projection of a coarse partition onto the finer level (Sec. 3). */
void or_project(uint32_t n, const uint32_t *cid, const uint32_t *coarse_part, uint32_t *part)
{
    for (uint32_t v = 0; v < n; ++v) part[v] = coarse_part[cid[v]];
}

/* ------------------------------------------------------------------------ */
/* Greedy initial partition (a simple deterministic method, as permitted for */
/* the coarsest level): BFS order, blocks filled to ceil(c(V)/k) in turn.     */
/* ------------------------------------------------------------------------ */
static int greedy_fill(const or_hg *h, uint32_t k, const int64_t *target, uint32_t *part);

int or_greedy_ip(const or_hg *h, uint32_t k, uint32_t *part)
{
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * k);
    const int64_t W = or_total_weight(h);
    for (uint32_t b = 0; b < k; ++b) T[b] = (W + (int64_t)k - 1) / (int64_t)k;
    int rc = greedy_fill(h, k, T, part);
    free(T);
    return rc;
}

/* The same fill with a weight target per block (block b is left once its
 * weight reaches target[b]); the bisections of R19 fill block 0 to its share
 * of the weight. */
int or_greedy_ip_targets(const or_hg *h, uint32_t k, const int64_t *target, uint32_t *part)
{
    return greedy_fill(h, k, target, part);
}

static int greedy_fill(const or_hg *h, uint32_t k, const int64_t *target, uint32_t *part)
{
    const uint32_t n = h->n;
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t *vis = (uint8_t *)calloc(n ? n : 1, 1);
    uint32_t head = 0, tail = 0, next_start = 0;
    while (tail < n) {
        while (vis[next_start]) ++next_start;
        vis[next_start] = 1;
        order[tail++] = next_start;
        while (head < tail) {
            uint32_t v = order[head++];
            for (uint32_t j = h->inc_off[v]; j < h->inc_off[v + 1]; ++j) {
                uint32_t e = h->inc[j];
                for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) {
                    uint32_t w = h->pins[q];
                    if (!vis[w]) { vis[w] = 1; order[tail++] = w; }
                }
            }
        }
    }
    uint32_t b = 0;
    int64_t cb = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = order[i];
        part[v] = b;
        cb += h->vwgt[v];
        if (cb >= target[b] && b + 1 < k) { ++b; cb = 0; }
    }
    free(order); free(vis);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Deterministic synchronous label propagation (Sec. 11).                    */
/* ------------------------------------------------------------------------ */

/* Longest feasible prefixes of one block pair by the two-pointer walk
 * (Sec. 11, reading R8): A = moves s->t, B = moves t->s, each already in
 * priority order; x = weight(A[0:i]) - weight(B[0:j]).  Feasible iff
 * -beta_s <= x <= beta_t.  The walk advances i while x <= 0 (i.e. while the
 * source block s receives at least as much as it gives) and j while x > 0,
 * taking the only remaining side once one sequence is exhausted.  Returns 1
 * and the last feasible visited state, or 0 (approve nothing). */
int or_select_pair(const int32_t *ca, uint32_t la, const int32_t *cb, uint32_t lb,
                   int64_t beta_s, int64_t beta_t, uint32_t *i_out, uint32_t *j_out)
{
    uint32_t i = 0, j = 0;
    int64_t sa = 0, sb = 0;
    int found = 0;
    *i_out = 0; *j_out = 0;
    for (;;) {
        int64_t x = sa - sb;
        if (-beta_s <= x && x <= beta_t) { found = 1; *i_out = i; *j_out = j; }
        if (i == la && j == lb) break;
        if (i == la) { sb += cb[j]; ++j; }
        else if (j == lb) { sa += ca[i]; ++i; }
        else if (x <= 0) { sa += ca[i]; ++i; }
        else { sb += cb[j]; ++j; }
    }
    if (!found) { *i_out = 0; *j_out = 0; }
    return found;
}

typedef struct { uint32_t s, t; int64_t g; uint32_t u; } or_move;

static int cmp_move(const void *a, const void *b)
{
    const or_move *x = (const or_move *)a, *y = (const or_move *)b;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    if (x->g != y->g) return x->g > y->g ? -1 : 1; /* gain descending */
    if (x->u != y->u) return x->u < y->u ? -1 : 1; /* node ID tie breaker */
    return 0;
}

/* Highest-gain move of u on the snapshot (part, bw): the block t != Pi[u]
 * with the largest positive gain among those that can take u without
 * exceeding L_max; ties to the smaller block (R10).  Returns OR_NONE if none. */
static uint32_t best_move(const or_hg *h, const uint32_t *part, const int64_t *bw,
                          const int64_t *lmax, uint32_t u, int64_t *aff, uint32_t *cnt,
                          uint32_t *blist, uint32_t *alist, int64_t *g_out)
{
    const uint32_t s = part[u];
    int64_t b_u = 0, w_inc = 0;
    uint32_t na = 0;
    for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
        uint32_t e = h->inc[j];
        uint32_t nb = 0;
        /* Phi(e, .) on the snapshot */
        for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) {
            uint32_t b = part[h->pins[q]];
            if (cnt[b]++ == 0) blist[nb++] = b;
        }
        w_inc += h->nwgt[e];
        if (cnt[s] == 1) b_u += h->nwgt[e];
        for (uint32_t q = 0; q < nb; ++q) {
            uint32_t t = blist[q];
            if (aff[t] == 0) alist[na++] = t;
            aff[t] += h->nwgt[e]; /* w({e in I(u): Phi(e,t) > 0}) */
            cnt[t] = 0;
        }
    }
    /* g(t) = b(u) - w({e in I(u): Phi(e,t) = 0}); only blocks with aff > 0 can be positive */
    uint32_t best = OR_NONE;
    int64_t bestg = 0;
    for (uint32_t q = 0; q < na; ++q) {
        uint32_t t = alist[q];
        int64_t g = b_u - (w_inc - aff[t]);
        aff[t] = 0;
        if (t == s || g <= 0) continue;
        if (bw[t] + h->vwgt[u] > lmax[t]) continue;
        if (g > bestg || (g == bestg && t < best)) { bestg = g; best = t; }
    }
    *g_out = bestg;
    return best;
}

/* The proposals of one LP sub-round (step 1 of Sec. 11's synchronous LP) on
 * the partition `part`: prop_t[u] = best target block or OR_NONE, prop_g[u]
 * its gain, for every node of sub-round s of round r.  Exposed for tests. */
static uint32_t lp_proposals_l(const or_hg *h, const or_params *P, uint32_t level, uint32_t r, uint32_t s,
                               const uint32_t *part, const int64_t *lmax_in, uint32_t *prop_t, int64_t *prop_g);

uint32_t or_lp_proposals(const or_hg *h, const or_params *P, uint32_t level, uint32_t r, uint32_t s,
                         const uint32_t *part, uint32_t *prop_t, int64_t *prop_g)
{
    return lp_proposals_l(h, P, level, r, s, part, NULL, prop_t, prop_g);
}

/* The same with per-block weight limits lmax[k]. */
uint32_t or_lp_proposals_limits(const or_hg *h, const or_params *P, uint32_t level, uint32_t r, uint32_t s,
                                const uint32_t *part, const int64_t *lmax, uint32_t *prop_t, int64_t *prop_g)
{
    return lp_proposals_l(h, P, level, r, s, part, lmax, prop_t, prop_g);
}

static uint32_t lp_proposals_l(const or_hg *h, const or_params *P, uint32_t level, uint32_t r, uint32_t s,
                               const uint32_t *part, const int64_t *lmax_in, uint32_t *prop_t, int64_t *prop_g)
{
    const uint32_t n = h->n, k = P->k;
    const int64_t W = or_total_weight(h);
    int64_t *lmax = (int64_t *)malloc(sizeof(int64_t) * k);
    for (uint32_t b = 0; b < k; ++b) lmax[b] = lmax_in ? lmax_in[b] : or_lmax(W, k, P->eps_num, P->eps_den);
    int64_t *bw = (int64_t *)malloc(sizeof(int64_t) * k);
    int64_t *aff = (int64_t *)calloc(k, sizeof(int64_t));
    uint32_t *cnt = (uint32_t *)calloc(k, sizeof(uint32_t));
    uint32_t *blist = (uint32_t *)malloc(sizeof(uint32_t) * k);
    uint32_t *alist = (uint32_t *)malloc(sizeof(uint32_t) * k);
    or_objective(h, k, part, bw);
    uint32_t np = 0;
    for (uint32_t u = 0; u < n; ++u) {
        prop_t[u] = OR_NONE;
        prop_g[u] = 0;
        if (or_hash(P->seed, 3, level, r, u) % P->lp_subrounds != s) continue;
        int64_t g;
        uint32_t t = best_move(h, part, bw, lmax, u, aff, cnt, blist, alist, &g);
        if (t == OR_NONE) continue;
        prop_t[u] = t;
        prop_g[u] = g;
        ++np;
    }
    free(lmax); free(bw); free(aff); free(cnt); free(blist); free(alist);
    return np;
}

/* LP refinement of one level.  part is refined in place; returns the
 * objective and block weights of the result.  lmax[b] is the weight limit of
 * block b: L_max for every block, or the per-side limits of a bisection of
 * the recursive bipartitioning (R19); the pair budgets of R9 take each
 * block's own limit. */
static int refine_lp_l(const or_hg *h, const or_params *P, uint32_t level, uint32_t *part, const int64_t *lmax,
                       int64_t *f_out, int64_t *block_w, uint32_t *rounds_out, uint64_t *moves_out)
{
    const uint32_t n = h->n, k = P->k;
    int64_t *bw = (int64_t *)malloc(sizeof(int64_t) * k);
    int64_t *aff = (int64_t *)calloc(k, sizeof(int64_t));
    uint32_t *cnt = (uint32_t *)calloc(k, sizeof(uint32_t));
    uint32_t *blist = (uint32_t *)malloc(sizeof(uint32_t) * k);
    uint32_t *alist = (uint32_t *)malloc(sizeof(uint32_t) * k);
    uint32_t *snap = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    or_move *M = (or_move *)malloc(sizeof(or_move) * (n ? n : 1));
    int32_t *ca = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *cb = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    uint32_t *pos_ab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k * k);
    uint32_t *len_ab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k * k);
    uint64_t total_moves = 0;
    uint32_t rounds = 0;
    or_objective(h, k, part, bw);

    for (uint32_t r = 0; r < P->lp_rounds; ++r) {
        uint64_t round_moves = 0;
        ++rounds;
        for (uint32_t sub = 0; sub < P->lp_subrounds; ++sub) {
            /* 1. highest-gain move of every node of this sub-round, on the snapshot */
            memcpy(snap, part, sizeof(uint32_t) * n);
            uint32_t nm = 0;
            for (uint32_t u = 0; u < n; ++u) {
                if (or_hash(P->seed, 3, level, r, u) % P->lp_subrounds != sub) continue;
                int64_t g;
                uint32_t t = best_move(h, snap, bw, lmax, u, aff, cnt, blist, alist, &g);
                if (t == OR_NONE) continue;
                M[nm].s = snap[u]; M[nm].t = t; M[nm].g = g; M[nm].u = u; ++nm;
            }
            /* 2. per block pair, sort by gain (node ID tie breaker) */
            qsort(M, nm, sizeof(or_move), cmp_move);
            for (size_t q = 0; q < (size_t)k * k; ++q) { len_ab[q] = 0; pos_ab[q] = 0; }
            for (uint32_t q = 0; q < nm; ++q) {
                size_t key = (size_t)M[q].s * k + M[q].t;
                if (len_ab[key] == 0) pos_ab[key] = q;
                len_ab[key]++;
            }
            /* 3. longest feasible prefixes, per-pair budget beta_b (R9) */
            uint64_t sub_moves = 0;
            for (uint32_t s = 0; s < k; ++s) {
                for (uint32_t t = s + 1; t < k; ++t) {
                    uint32_t la = len_ab[(size_t)s * k + t], lb = len_ab[(size_t)t * k + s];
                    if (la == 0 && lb == 0) continue;
                    uint32_t pa = pos_ab[(size_t)s * k + t], pb = pos_ab[(size_t)t * k + s];
                    for (uint32_t q = 0; q < la; ++q) ca[q] = h->vwgt[M[pa + q].u];
                    for (uint32_t q = 0; q < lb; ++q) cb[q] = h->vwgt[M[pb + q].u];
                    int64_t beta_s = floor_div(lmax[s] - bw[s], (int64_t)k - 1);
                    int64_t beta_t = floor_div(lmax[t] - bw[t], (int64_t)k - 1);
                    uint32_t ii, jj;
                    or_select_pair(ca, la, cb, lb, beta_s, beta_t, &ii, &jj);
                    for (uint32_t q = 0; q < ii; ++q) { part[M[pa + q].u] = t; }
                    for (uint32_t q = 0; q < jj; ++q) { part[M[pb + q].u] = s; }
                    sub_moves += ii + jj;
                }
            }
            /* 4. apply: block weights of the new assignment */
            if (sub_moves) {
                for (uint32_t b = 0; b < k; ++b) bw[b] = 0;
                for (uint32_t v = 0; v < n; ++v) bw[part[v]] += h->vwgt[v];
            }
            round_moves += sub_moves;
        }
        total_moves += round_moves;
        if (round_moves == 0) break;
    }
    int64_t f = or_objective(h, k, part, block_w);
    if (f_out) *f_out = f;
    if (rounds_out) *rounds_out = rounds;
    if (moves_out) *moves_out = total_moves;
    free(bw); free(aff); free(cnt); free(blist); free(alist); free(snap); free(M); free(ca); free(cb); free(pos_ab); free(len_ab);
    return OR_OK;
}

int or_refine_lp(const or_hg *h, const or_params *P, uint32_t level, uint32_t *part,
                 int64_t *f_out, int64_t *block_w, uint32_t *rounds_out, uint64_t *moves_out)
{
    int64_t *lmax = (int64_t *)malloc(sizeof(int64_t) * P->k);
    const int64_t L = or_lmax(or_total_weight(h), P->k, P->eps_num, P->eps_den);
    for (uint32_t b = 0; b < P->k; ++b) lmax[b] = L;
    int rc = refine_lp_l(h, P, level, part, lmax, f_out, block_w, rounds_out, moves_out);
    free(lmax);
    return rc;
}

/* LP with explicit per-block weight limits (the bisections of R19). */
int or_refine_lp_limits(const or_hg *h, const or_params *P, uint32_t level, uint32_t *part, const int64_t *lmax,
                        int64_t *f_out, int64_t *block_w, uint32_t *rounds_out, uint64_t *moves_out)
{
    return refine_lp_l(h, P, level, part, lmax, f_out, block_w, rounds_out, moves_out);
}

/* ------------------------------------------------------------------------ */
/* Multilevel driver (Alg. 1 of the paper, with the SDet-style components).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t n, m, p;
    uint32_t *pin_off, *pins, *inc_off, *inc, *cid;
    int32_t *vwgt, *nwgt;
} or_level;

static or_hg view(const or_level *L)
{
    or_hg h;
    h.n = L->n; h.m = L->m; h.p = L->p;
    h.pin_off = L->pin_off; h.pins = L->pins; h.inc_off = L->inc_off; h.inc = L->inc;
    h.vwgt = L->vwgt; h.nwgt = L->nwgt;
    return h;
}

/* ------------------------------------------------------------------------ */
/* Community detection (Sec. 4.3) by the deterministic Louvain method       */
/* (Sec. 11) on the bipartite graph representation G_x of the hypergraph.   */
/* Readings: R16 (edge weights), R17 (synchronous local moving and its      */
/* integer modularity comparison), R18 (levels).                             */
/* ------------------------------------------------------------------------ */
#define OR_LV_ROUNDS 5      /* local moving rounds per level            */
#define OR_LV_SUBROUNDS 5   /* sub-rounds per round                     */
#define OR_LV_LEVELS 16     /* contraction levels at most               */

/* G_x as a two-pin hypergraph: node u < n is vertex u, node n + e is net e;
 * edge j (one per pin, in pin order) joins the pin's vertex and net node and
 * weighs w(e) (R16).  Node weights are the volumes (sums of incident edge
 * weights): vol(u) = sum of w(e) over the nets of u, vol(n+e) = |e| w(e).
 * Arrays sized pin_off[p+1], pins[2p], inc_off[n+m+1], inc[2p], vwgt[n+m],
 * nwgt[p].  The total volume must stay below 2^31 (OR_E_INVALID). */
int or_bipartite(const or_hg *h, uint32_t *pin_off, uint32_t *pins, uint32_t *inc_off, uint32_t *inc,
                 int32_t *vwgt, int32_t *nwgt)
{
    const uint32_t n = h->n, m = h->m, p = h->p;
    int64_t total = 0;
    for (uint32_t e = 0; e < m; ++e)
        total += 2 * (int64_t)(h->pin_off[e + 1] - h->pin_off[e]) * h->nwgt[e];
    if (total >= ((int64_t)1 << 31)) return OR_E_INVALID;
    uint32_t *cursor = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!cursor) return OR_E_NOMEM;
    for (uint32_t u = 0; u < n; ++u) { cursor[u] = h->inc_off[u]; vwgt[u] = 0; }
    for (uint32_t j = 0; j <= p; ++j) pin_off[j] = 2 * j;
    for (uint32_t u = 0; u <= n; ++u) inc_off[u] = h->inc_off[u];
    for (uint32_t e = 0; e < m; ++e) {
        inc_off[n + e + 1] = p + h->pin_off[e + 1];
        vwgt[n + e] = (int32_t)((h->pin_off[e + 1] - h->pin_off[e]) * (int64_t)h->nwgt[e]);
        for (uint32_t j = h->pin_off[e]; j < h->pin_off[e + 1]; ++j) {
            const uint32_t u = h->pins[j];
            pins[2 * j] = u;
            pins[2 * j + 1] = n + e;
            nwgt[j] = h->nwgt[e];
            inc[cursor[u]++] = j;     /* nets ascending, so edges ascending per vertex */
            inc[p + j] = j;
            vwgt[u] += h->nwgt[e];
        }
    }
    free(cursor);
    return OR_OK;
}

/* One sub-round (r, s) of synchronous local moving (R17) on a graph g (a
 * two-pin hypergraph; vwgt = volumes, nwgt = edge weights) at Louvain level
 * `level`.  The nodes x with H(seed, 4, level, r, x) mod S = s decide on the
 * state at the start of the sub-round: with m_2 = the total volume (twice the
 * edge weight), A = comm[x], w(x, C) = the weight of x's edges into C and
 * vol(C) = cvol[C], the move to C != A changes the modularity by
 * [score(C) - score(A)] / (m_2^2 / 2) where score(C) = m_2 w(x, C) - vol(x)
 * vol(C) and score(A) = m_2 w(x, A) - vol(x) (vol(A) - vol(x)).  The best C
 * among x's neighbour communities (largest score, then smallest ID) is
 * taken when its score exceeds score(A).  All moves of the sub-round are then
 * applied and the volumes updated.  Returns the number of moves. */
uint32_t or_louvain_subround(const or_hg *g, uint64_t seed, uint32_t level, uint32_t r, uint32_t s,
                             uint32_t *comm, int64_t *cvol)
{
    const uint32_t N = g->n;
    int64_t m2 = 0;
    for (uint32_t x = 0; x < N; ++x) m2 += g->vwgt[x];
    int64_t *acc = (int64_t *)calloc(N ? N : 1, sizeof(int64_t));
    uint32_t *touched = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    uint32_t *dec = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    for (uint32_t x = 0; x < N; ++x) {
        dec[x] = OR_NONE;
        if (or_hash(seed, 4, level, r, x) % OR_LV_SUBROUNDS != s) continue;
        const uint32_t A = comm[x];
        const int64_t vx = g->vwgt[x];
        uint32_t nt = 0;
        for (uint32_t j = g->inc_off[x]; j < g->inc_off[x + 1]; ++j) {
            const uint32_t e = g->inc[j];
            const uint32_t a = g->pins[g->pin_off[e]], b = g->pins[g->pin_off[e] + 1];
            const uint32_t c = comm[a == x ? b : a];
            if (acc[c] == 0) touched[nt++] = c;   /* every edge weight is >= 1 */
            acc[c] += g->nwgt[e];
        }
        const int64_t score_a = m2 * acc[A] - vx * (cvol[A] - vx);
        uint32_t best = OR_NONE;
        int64_t best_s = 0;
        for (uint32_t q = 0; q < nt; ++q) {
            const uint32_t c = touched[q];
            if (c == A) continue;
            const int64_t sc = m2 * acc[c] - vx * cvol[c];
            if (best == OR_NONE || sc > best_s || (sc == best_s && c < best)) { best = c; best_s = sc; }
        }
        for (uint32_t q = 0; q < nt; ++q) acc[touched[q]] = 0;
        if (best != OR_NONE && best_s > score_a) dec[x] = best;
    }
    uint32_t moves = 0;
    for (uint32_t x = 0; x < N; ++x) {
        if (dec[x] == OR_NONE) continue;
        cvol[comm[x]] -= g->vwgt[x];
        cvol[dec[x]] += g->vwgt[x];
        comm[x] = dec[x];
        ++moves;
    }
    free(acc); free(touched); free(dec);
    return moves;
}

/* Local moving of one level from singleton communities: rounds of
 * OR_LV_SUBROUNDS sub-rounds, at most OR_LV_ROUNDS, until a round moves no
 * node (R17).  comm[x] receives a node ID per community; returns the moves. */
uint32_t or_louvain_level(const or_hg *g, uint64_t seed, uint32_t level, uint32_t *comm, uint32_t *rounds_out)
{
    const uint32_t N = g->n;
    int64_t *cvol = (int64_t *)malloc(sizeof(int64_t) * (N ? N : 1));
    for (uint32_t x = 0; x < N; ++x) { comm[x] = x; cvol[x] = g->vwgt[x]; }
    uint32_t total = 0, r = 0;
    while (r < OR_LV_ROUNDS) {
        uint32_t mv = 0;
        for (uint32_t s = 0; s < OR_LV_SUBROUNDS; ++s) mv += or_louvain_subround(g, seed, level, r, s, comm, cvol);
        ++r;
        total += mv;
        if (mv == 0) break;
    }
    free(cvol);
    if (rounds_out) *rounds_out = r;
    return total;
}

/* Communities of the vertices (Sec. 4.3, R18).  Level 0 is G_x.  After the
 * local moving of a level, each community is contracted into one node (its
 * representative is its smallest node ID; the contraction of Sec. 4.2 drops
 * the self-loops and merges parallel edges, and the node weights -- the
 * volumes -- add up), and the next level starts again from singletons.  The
 * levels stop when a level moves no node, when a contraction does not shrink
 * the graph, or after OR_LV_LEVELS levels.  comm[u] (u < n) is the node of
 * the last level that holds u. */
int or_communities(const or_hg *h, uint64_t seed, uint32_t *comm_out, uint32_t *levels_out)
{
    const uint32_t n = h->n, m = h->m, p = h->p, N = n + m;
    or_level G[2];
    for (int b = 0; b < 2; ++b) {
        G[b].pin_off = (uint32_t *)malloc(sizeof(uint32_t) * (p + 1));
        G[b].pins = (uint32_t *)malloc(sizeof(uint32_t) * (2 * (size_t)p + 1));
        G[b].inc_off = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
        G[b].inc = (uint32_t *)malloc(sizeof(uint32_t) * (2 * (size_t)p + 1));
        G[b].vwgt = (int32_t *)malloc(sizeof(int32_t) * (N ? N : 1));
        G[b].nwgt = (int32_t *)malloc(sizeof(int32_t) * (p ? p : 1));
        G[b].cid = NULL;
    }
    uint32_t *map = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    uint32_t *comm = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    uint32_t *minid = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    uint32_t *rep = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    uint32_t *cid = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
    int rc = or_bipartite(h, G[0].pin_off, G[0].pins, G[0].inc_off, G[0].inc, G[0].vwgt, G[0].nwgt);
    uint32_t levels = 0;
    if (rc == OR_OK) {
        G[0].n = N; G[0].m = p; G[0].p = 2 * p;
        for (uint32_t x = 0; x < N; ++x) map[x] = x;
        int cur = 0;
        for (uint32_t level = 0; level < OR_LV_LEVELS; ++level) {
            or_hg g = view(&G[cur]);
            if (or_louvain_level(&g, seed, level, comm, NULL) == 0) break;
            for (uint32_t x = 0; x < g.n; ++x) minid[x] = OR_NONE;
            for (uint32_t x = 0; x < g.n; ++x)
                if (minid[comm[x]] == OR_NONE) minid[comm[x]] = x;
            for (uint32_t x = 0; x < g.n; ++x) rep[x] = minid[comm[x]];
            or_level *nx = &G[1 - cur];
            uint32_t dims[3];
            or_contract(&g, rep, cid, dims, nx->pin_off, nx->pins, nx->inc_off, nx->inc, nx->vwgt, nx->nwgt);
            nx->n = dims[0]; nx->m = dims[1]; nx->p = dims[2];
            for (uint32_t x = 0; x < N; ++x) map[x] = cid[map[x]];
            ++levels;
            cur = 1 - cur;
            if (nx->n == g.n) break;
        }
        for (uint32_t u = 0; u < n; ++u) comm_out[u] = map[u];
    }
    if (levels_out) *levels_out = levels;
    for (int b = 0; b < 2; ++b) {
        free(G[b].pin_off); free(G[b].pins); free(G[b].inc_off); free(G[b].inc); free(G[b].vwgt); free(G[b].nwgt);
    }
    free(map); free(comm); free(minid); free(rep); free(cid);
    return rc;
}


/* Partition: coarsen while n > 160k and the pass shrinks the level by more
 * than 1% (Sec. 4.1 contraction limits), greedy initial partition on the
 * coarsest level, then project + LP per level (LP also on the coarsest level,
 * R11).  levels_out gets the number of contractions performed. */
int or_rb_ip(const or_hg *h, const or_params *P, uint32_t *part);

/* The multilevel cycle: coarsen while n > 160k and the pass shrinks the
 * level by more than 1% (Sec. 4.1 contraction limits), initial partition of
 * the coarsest level, then project + LP per level (LP also on the coarsest
 * level, R11).  lmax (k entries, or NULL for L_max on every block) and
 * target (the fill targets of the greedy initial partition, or NULL for
 * ceil(c(V)/k)) are set by the bisections of R19.  levels_out gets the number
 * of contractions performed. */
static int multilevel(const or_hg *h0, const or_params *P, const int64_t *lmax_in, const int64_t *target,
                      uint32_t *part, int64_t *f_out, uint32_t *levels_out)
{
    const uint32_t MAXL = 4096;
    or_level *L = (or_level *)calloc(MAXL, sizeof(or_level));
    uint32_t nl = 0;
    const or_hg *cur = h0;
    or_hg tmp;
    uint32_t *rep = (uint32_t *)malloc(sizeof(uint32_t) * (h0->n ? h0->n : 1));
    /* community-aware coarsening (Sec. 4.3): the communities of the input,
     * carried to every coarse level through the contraction map */
    uint32_t *comm = NULL, *ccomm = NULL;
    if (P->community) {
        comm = (uint32_t *)malloc(sizeof(uint32_t) * (h0->n ? h0->n : 1));
        ccomm = (uint32_t *)malloc(sizeof(uint32_t) * (h0->n ? h0->n : 1));
        if (or_communities(h0, P->seed, comm, NULL) != OR_OK) { free(L); free(rep); free(comm); free(ccomm); return OR_E_INVALID; }
    }
    for (;;) {
        if (!((uint64_t)cur->n > (uint64_t)P->limit_factor * P->k)) break;
        uint32_t cnt;
        cluster_pass(cur, P, nl, comm, rep, &cnt, NULL);
        if ((uint64_t)100 * (cur->n - cnt) <= (uint64_t)cur->n) break;
        or_level *N = &L[nl];
        N->cid = (uint32_t *)malloc(sizeof(uint32_t) * (cur->n ? cur->n : 1));
        N->pin_off = (uint32_t *)malloc(sizeof(uint32_t) * (cur->m + 1));
        N->pins = (uint32_t *)malloc(sizeof(uint32_t) * (cur->p ? cur->p : 1));
        N->inc_off = (uint32_t *)malloc(sizeof(uint32_t) * (cur->n + 1));
        N->inc = (uint32_t *)malloc(sizeof(uint32_t) * (cur->p ? cur->p : 1));
        N->vwgt = (int32_t *)malloc(sizeof(int32_t) * (cur->n ? cur->n : 1));
        N->nwgt = (int32_t *)malloc(sizeof(int32_t) * (cur->m ? cur->m : 1));
        uint32_t dims[3];
        or_contract(cur, rep, N->cid, dims, N->pin_off, N->pins, N->inc_off, N->inc, N->vwgt, N->nwgt);
        N->n = dims[0]; N->m = dims[1]; N->p = dims[2];
        if (comm) {
            for (uint32_t v = 0; v < cur->n; ++v) ccomm[N->cid[v]] = comm[v];
            memcpy(comm, ccomm, sizeof(uint32_t) * N->n);
        }
        ++nl;
        tmp = view(N);
        cur = &tmp;
        if (nl == MAXL) break;
    }
    /* initial partition of the coarsest level and LP on it */
    const uint32_t k = P->k;
    int64_t *lmax = (int64_t *)malloc(sizeof(int64_t) * k);
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * k);
    const int64_t W = or_total_weight(h0);
    for (uint32_t b = 0; b < k; ++b) {
        lmax[b] = lmax_in ? lmax_in[b] : or_lmax(W, k, P->eps_num, P->eps_den);
        T[b] = target ? target[b] : (W + (int64_t)k - 1) / (int64_t)k;
    }
    uint32_t *cp = (uint32_t *)malloc(sizeof(uint32_t) * (cur->n ? cur->n : 1));
    if (P->ip == 1) or_rb_ip(cur, P, cp);
    else greedy_fill(cur, k, T, cp);
    int64_t f;
    refine_lp_l(cur, P, nl, cp, lmax, &f, NULL, NULL, NULL);
    /* uncoarsening */
    for (int l = (int)nl - 1; l >= 0; --l) {
        or_hg fine = (l == 0) ? *h0 : view(&L[l - 1]);
        uint32_t *fp = (uint32_t *)malloc(sizeof(uint32_t) * (fine.n ? fine.n : 1));
        or_project(fine.n, L[l].cid, cp, fp);
        free(cp);
        cp = fp;
        refine_lp_l(&fine, P, (uint32_t)l, cp, lmax, &f, NULL, NULL, NULL);
    }
    memcpy(part, cp, sizeof(uint32_t) * h0->n);
    *f_out = f;
    if (levels_out) *levels_out = nl;
    for (uint32_t l = 0; l < nl; ++l) {
        free(L[l].cid); free(L[l].pin_off); free(L[l].pins); free(L[l].inc_off);
        free(L[l].inc); free(L[l].vwgt); free(L[l].nwgt);
    }
    free(L); free(rep); free(cp); free(comm); free(ccomm); free(lmax); free(T);
    return OR_OK;
}

int or_partition(const or_hg *h0, const or_params *P, uint32_t *part, int64_t *f_out, uint32_t *levels_out)
{
    return multilevel(h0, P, NULL, NULL, part, f_out, levels_out);
}

/* ------------------------------------------------------------------------ */
/* Recursive bipartitioning initial partition (Sec. 5, Eq. 1; reading R19).  */
/* ------------------------------------------------------------------------ */

/* Limits and fill targets of the bisection of a subhypergraph of weight Wsub
 * that gets kk blocks, in a partition of a hypergraph of weight Wtot into
 * ktot blocks: side 0 gets ceil(kk/2) blocks, side 1 floor(kk/2).  The
 * imbalance of the bisection is eps' of Eq. 1, computed in IEEE double with
 * the C library's pow; side i's target is ceil(Wsub k_i / kk) and its limit
 * floor((1 + eps') target_i). */
void or_rb_limits(int64_t Wtot, uint32_t ktot, uint32_t eps_num, uint32_t eps_den, int64_t Wsub, uint32_t kk,
                  int64_t *L, int64_t *T)
{
    const uint32_t ks[2] = {(kk + 1) / 2, kk / 2};
    uint32_t lg = 0;
    while ((1u << lg) < kk) ++lg; /* ceil(log2 kk) */
    const double eps = (double)eps_num / (double)eps_den;
    const double base = (1.0 + eps) * ((double)Wtot / (double)ktot) * ((double)kk / (double)Wsub);
    const double epsp = pow(base, 1.0 / (double)lg) - 1.0;
    for (int i = 0; i < 2; ++i) {
        T[i] = (Wsub * (int64_t)ks[i] + (int64_t)kk - 1) / (int64_t)kk;
        L[i] = (int64_t)floor((1.0 + epsp) * (double)T[i]);
    }
}

/* Subhypergraph H[V'] of Sec. 2 for V' = the vertices with part[v] == side:
 * its vertices renumbered in ascending ID, every net with a pin in V'
 * restricted to those pins (ascending net ID, weights kept, single-pin nets
 * included as the definition has them).  vmap[i] = the vertex of h that new
 * vertex i stands for.  Arrays are malloc'ed into S. */
int or_subhypergraph(const or_hg *h, const uint32_t *part, uint32_t side, uint32_t *dims, uint32_t *pin_off,
                     uint32_t *pins, uint32_t *inc_off, uint32_t *inc, int32_t *vwgt, int32_t *nwgt, uint32_t *vmap)
{
    const uint32_t n = h->n, m = h->m;
    uint32_t *nid = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t n2 = 0;
    for (uint32_t v = 0; v < n; ++v) {
        nid[v] = OR_NONE;
        if (part[v] == side) { nid[v] = n2; vmap[n2] = v; vwgt[n2] = h->vwgt[v]; ++n2; }
    }
    uint32_t m2 = 0, p2 = 0;
    pin_off[0] = 0;
    for (uint32_t e = 0; e < m; ++e) {
        const uint32_t b = p2;
        for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q)
            if (nid[h->pins[q]] != OR_NONE) pins[p2++] = nid[h->pins[q]];
        if (p2 == b) continue;
        nwgt[m2] = h->nwgt[e];
        pin_off[++m2] = p2;
    }
    /* incidence lists: nets ascending per vertex */
    for (uint32_t v = 0; v <= n2; ++v) inc_off[v] = 0;
    for (uint32_t q = 0; q < p2; ++q) inc_off[pins[q] + 1]++;
    for (uint32_t v = 0; v < n2; ++v) inc_off[v + 1] += inc_off[v];
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (n2 ? n2 : 1));
    for (uint32_t v = 0; v < n2; ++v) cur[v] = inc_off[v];
    for (uint32_t e = 0; e < m2; ++e)
        for (uint32_t q = pin_off[e]; q < pin_off[e + 1]; ++q) inc[cur[pins[q]]++] = e;
    dims[0] = n2; dims[1] = m2; dims[2] = p2;
    free(nid); free(cur);
    return OR_OK;
}

/* The bisection of one subhypergraph: the multilevel cycle with k = 2 (no
 * community detection, greedy fill at the bottom), block i limited to L[i],
 * block 0 filled to T[0]. */
int or_bisect(const or_hg *h, const or_params *P, const int64_t *L, const int64_t *T, uint32_t *part)
{
    or_params P2 = *P;
    P2.k = 2;
    P2.community = 0;
    P2.ip = 0;
    int64_t f;
    return multilevel(h, &P2, L, T, part, &f, NULL);
}

static void rb(const or_hg *h, const or_params *P, int64_t Wtot, uint32_t ktot, uint32_t kk, uint32_t b0,
               const uint32_t *vmap, uint32_t *out)
{
    const uint32_t n = h->n;
    if (n == 0) return;
    if (kk == 1) {
        for (uint32_t v = 0; v < n; ++v) out[vmap[v]] = b0;
        return;
    }
    int64_t L[2], T[2];
    or_rb_limits(Wtot, ktot, P->eps_num, P->eps_den, or_total_weight(h), kk, L, T);
    uint32_t *bp = (uint32_t *)malloc(sizeof(uint32_t) * n);
    or_bisect(h, P, L, T, bp);
    const uint32_t ks[2] = {(kk + 1) / 2, kk / 2};
    for (uint32_t side = 0; side < 2; ++side) {
        or_level S;
        uint32_t dims[3];
        S.pin_off = (uint32_t *)malloc(sizeof(uint32_t) * (h->m + 1));
        S.pins = (uint32_t *)malloc(sizeof(uint32_t) * (h->p ? h->p : 1));
        S.inc_off = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
        S.inc = (uint32_t *)malloc(sizeof(uint32_t) * (h->p ? h->p : 1));
        S.vwgt = (int32_t *)malloc(sizeof(int32_t) * n);
        S.nwgt = (int32_t *)malloc(sizeof(int32_t) * (h->m ? h->m : 1));
        S.cid = NULL;
        uint32_t *smap = (uint32_t *)malloc(sizeof(uint32_t) * n);
        or_subhypergraph(h, bp, side, dims, S.pin_off, S.pins, S.inc_off, S.inc, S.vwgt, S.nwgt, smap);
        S.n = dims[0]; S.m = dims[1]; S.p = dims[2];
        for (uint32_t i = 0; i < S.n; ++i) smap[i] = vmap[smap[i]];
        or_hg sh = view(&S);
        rb(&sh, P, Wtot, ktot, ks[side], side == 0 ? b0 : b0 + ks[0], smap, out);
        free(S.pin_off); free(S.pins); free(S.inc_off); free(S.inc); free(S.vwgt); free(S.nwgt); free(smap);
    }
    free(bp);
}

/* Recursive bipartitioning (Sec. 5, R19): the k-way initial partition of h
 * by bisections with the imbalance of Eq. 1; side 0 of a bisection into kk
 * blocks takes blocks b0 .. b0 + ceil(kk/2) - 1, side 1 the rest. */
int or_rb_ip(const or_hg *h, const or_params *P, uint32_t *part)
{
    uint32_t *vmap = (uint32_t *)malloc(sizeof(uint32_t) * (h->n ? h->n : 1));
    for (uint32_t v = 0; v < h->n; ++v) vmap[v] = v;
    rb(h, P, or_total_weight(h), P->k, P->k, 0, vmap, part);
    free(vmap);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Gain table (Sec. 6.2): benefit b(u) = w({e in I(u): Phi(e, Pi[u]) = 1})  */
/* and penalty p(u, V_t) = w({e in I(u): Phi(e, V_t) = 0}), so that         */
/* g_u(t) = b(u) - p(u, V_t).  pen is row major, n rows of k entries.       */
/* ------------------------------------------------------------------------ */
int or_gain_table(const or_hg *h, uint32_t k, const uint32_t *part, int64_t *ben, int64_t *pen)
{
    uint32_t *cnt = (uint32_t *)calloc(k, sizeof(uint32_t));
    if (!cnt) return OR_E_NOMEM;
    for (uint32_t u = 0; u < h->n; ++u) {
        ben[u] = 0;
        for (uint32_t t = 0; t < k; ++t) pen[(size_t)u * k + t] = 0;
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            uint32_t e = h->inc[j];
            for (uint32_t t = 0; t < k; ++t) cnt[t] = 0;
            for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) cnt[part[h->pins[q]]]++;
            if (cnt[part[u]] == 1) ben[u] += h->nwgt[e];
            for (uint32_t t = 0; t < k; ++t)
                if (cnt[t] == 0) pen[(size_t)u * k + t] += h->nwgt[e];
        }
    }
    free(cnt);
    return OR_OK;
}

/* Moves u_i -> t_i (i = 0..l-1, every node at most once) applied one after
 * the other to part, with the update rules of Sec. 6.2 on the gain table
 * after each move: with Phi updated for the move (Phi(e, s) - 1 and
 * Phi(e, t) + 1 for every e in I(u)), a penalty for s is added for every pin
 * of e when Phi(e, s) reaches 0, a benefit is added to the pin left alone in
 * s when Phi(e, s) reaches 1, the penalty for t is taken back from every pin
 * when Phi(e, t) reaches 1, and the benefit of the pin that was alone in t is
 * taken back when Phi(e, t) reaches 2.  As in the paper, the benefits of the
 * moved nodes are recomputed afterwards (their block changed).  part, ben and
 * pen are updated in place. */
int or_gain_table_moves(const or_hg *h, uint32_t k, uint32_t *part, const uint32_t *mu, const uint32_t *mt,
                        uint32_t l, int64_t *ben, int64_t *pen)
{
    const uint32_t m = h->m;
    uint32_t *phi = (uint32_t *)calloc((size_t)(m ? m : 1) * k, sizeof(uint32_t));
    uint8_t *moved = (uint8_t *)calloc(h->n ? h->n : 1, 1);
    if (!phi || !moved) return OR_E_NOMEM;
    for (uint32_t e = 0; e < m; ++e)
        for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) phi[(size_t)e * k + part[h->pins[q]]]++;
    for (uint32_t i = 0; i < l; ++i) {
        const uint32_t u = mu[i], s = part[u], t = mt[i];
        if (s == t) continue;
        part[u] = t;
        moved[u] = 1;
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            const uint32_t e = h->inc[j];
            const int64_t w = h->nwgt[e];
            const uint32_t ps = --phi[(size_t)e * k + s];
            const uint32_t pt = ++phi[(size_t)e * k + t];
            for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) {
                const uint32_t v = h->pins[q];
                if (ps == 0) pen[(size_t)v * k + s] += w;
                if (ps == 1 && part[v] == s) ben[v] += w;
                if (pt == 1) pen[(size_t)v * k + t] -= w;
                if (pt == 2 && part[v] == t) ben[v] -= w;
            }
        }
    }
    for (uint32_t u = 0; u < h->n; ++u) {
        if (!moved[u]) continue;
        ben[u] = 0;
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            const uint32_t e = h->inc[j];
            if (phi[(size_t)e * k + part[u]] == 1) ben[u] += h->nwgt[e];
        }
    }
    free(phi); free(moved);
    return OR_OK;
}

/* Gains of a move sequence (Sec. 6.3): g_i = f(Pi_{i-1}) - f(Pi_i), the
 * change of the connectivity objective made by move i when the moves are
 * performed in the order given, starting from part (unchanged here).  Each
 * move u_i -> t_i, every node moved at most once.  Computed by performing
 * the moves one after the other: a net leaves block s when its last pin in s
 * moves out (+w), and enters block t when its first pin arrives (-w). */
int or_gain_recalc(const or_hg *h, uint32_t k, const uint32_t *part, const uint32_t *mu, const uint32_t *mt,
                   uint32_t l, int64_t *g)
{
    const uint32_t m = h->m;
    uint32_t *phi = (uint32_t *)calloc((size_t)(m ? m : 1) * k, sizeof(uint32_t));
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (h->n ? h->n : 1));
    if (!phi || !cur) return OR_E_NOMEM;
    memcpy(cur, part, sizeof(uint32_t) * h->n);
    for (uint32_t e = 0; e < m; ++e)
        for (uint32_t q = h->pin_off[e]; q < h->pin_off[e + 1]; ++q) phi[(size_t)e * k + cur[h->pins[q]]]++;
    for (uint32_t i = 0; i < l; ++i) {
        const uint32_t u = mu[i], s = cur[u], t = mt[i];
        g[i] = 0;
        if (s == t) continue;
        cur[u] = t;
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            const uint32_t e = h->inc[j];
            if (--phi[(size_t)e * k + s] == 0) g[i] += h->nwgt[e];
            if (++phi[(size_t)e * k + t] == 1) g[i] -= h->nwgt[e];
        }
    }
    free(phi); free(cur);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Graphs (Sec. 10): every net has two pins.  The gain of moving u to V_t   */
/* is w(u, V_t) - w(u, V_Pi[u]) (external minus internal edge weight), read */
/* from one adjacency array: adj[j] is the other endpoint of the j-th edge  */
/* of u (in the order of u's incident nets), adjw[j] its weight.            */
/* ------------------------------------------------------------------------ */

/* Builds the adjacency array of a hypergraph whose nets all have two pins;
 * returns OR_E_INVALID if some net does not. */
int or_graph_adjacency(const or_hg *h, uint32_t *adj, int32_t *adjw)
{
    for (uint32_t e = 0; e < h->m; ++e)
        if (h->pin_off[e + 1] - h->pin_off[e] != 2) return OR_E_INVALID;
    for (uint32_t u = 0; u < h->n; ++u)
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            uint32_t e = h->inc[j];
            uint32_t a = h->pins[h->pin_off[e]], b = h->pins[h->pin_off[e] + 1];
            adj[j] = (a == u) ? b : a;
            adjw[j] = h->nwgt[e];
        }
    return OR_OK;
}

/* w(u, V_t) - w(u, V_Pi[u]) from the adjacency array. */
int64_t or_graph_gain(const or_hg *h, const uint32_t *adj, const int32_t *adjw, const uint32_t *part,
                      uint32_t u, uint32_t t)
{
    int64_t to_t = 0, internal = 0;
    for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
        if (part[adj[j]] == t) to_t += adjw[j];
        if (part[adj[j]] == part[u]) internal += adjw[j];
    }
    return to_t - internal;
}

/* Edge cut: the total weight of edges whose endpoints lie in different blocks. */
int64_t or_graph_cut(const or_hg *h, const uint32_t *part)
{
    int64_t c = 0;
    for (uint32_t e = 0; e < h->m; ++e)
        if (part[h->pins[h->pin_off[e]]] != part[h->pins[h->pin_off[e] + 1]]) c += h->nwgt[e];
    return c;
}

/* Graph gain table (Sec. 10): omega[u * k + i] = w(u, V_i), the total weight
 * of u's edges whose other endpoint lies in block i, summed over the
 * adjacency from the definition. */
int or_graph_gain_table(const or_hg *h, uint32_t k, const uint32_t *part, int64_t *omega)
{
    for (uint32_t e = 0; e < h->m; ++e)
        if (h->pin_off[e + 1] - h->pin_off[e] != 2) return OR_E_INVALID;
    memset(omega, 0, sizeof(int64_t) * (size_t)h->n * k);
    for (uint32_t u = 0; u < h->n; ++u)
        for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
            const uint32_t e = h->inc[j];
            const uint32_t a = h->pins[h->pin_off[e]], b = h->pins[h->pin_off[e] + 1];
            const uint32_t v = (a == u) ? b : a;
            omega[(size_t)u * k + part[v]] += h->nwgt[e];
        }
    return OR_OK;
}

/* A batch of moves on a graph (Sec. 10), made one after the other in the
 * order given, every node at most once.  Moving u from V_s to V_t adds w(u, v)
 * to w(v, V_t) and subtracts it from w(v, V_s) for every neighbour v (when
 * omega is not NULL), then sets Pi[u] = t.  The attributed gain of the move
 * (when gain is not NULL) sums, over the edges {u, v} of u, +w(e) for an edge
 * that stops being cut and -w(e) for one that becomes cut, with v in the
 * block it holds when u moves (reading R15: an edge whose state does not
 * change is attributed nothing).  A move to the node's own block is no move
 * (gain 0).  Invalid moves (node or block out of range, a node listed twice)
 * are rejected before anything changes. */
int or_graph_moves(const or_hg *h, uint32_t k, uint32_t *part, const uint32_t *mu, const uint32_t *mt,
                   uint32_t l, int64_t *omega, int64_t *gain)
{
    for (uint32_t e = 0; e < h->m; ++e)
        if (h->pin_off[e + 1] - h->pin_off[e] != 2) return OR_E_INVALID;
    uint8_t *seen = (uint8_t *)calloc(h->n ? h->n : 1, 1);
    if (!seen) return OR_E_NOMEM;
    for (uint32_t i = 0; i < l; ++i) {
        if (mu[i] >= h->n || mt[i] >= k || seen[mu[i]]) { free(seen); return OR_E_INVALID; }
        seen[mu[i]] = 1;
    }
    free(seen);
    for (uint32_t i = 0; i < l; ++i) {
        const uint32_t u = mu[i], s = part[u], t = mt[i];
        int64_t g = 0;
        if (s != t) {
            for (uint32_t j = h->inc_off[u]; j < h->inc_off[u + 1]; ++j) {
                const uint32_t e = h->inc[j];
                const uint32_t a = h->pins[h->pin_off[e]], b = h->pins[h->pin_off[e] + 1];
                const uint32_t v = (a == u) ? b : a;
                const int64_t w = h->nwgt[e];
                const int was_cut = part[v] != s, now_cut = part[v] != t;
                if (was_cut && !now_cut) g += w;
                if (!was_cut && now_cut) g -= w;
                if (omega) {
                    omega[(size_t)v * k + t] += w;
                    omega[(size_t)v * k + s] -= w;
                }
            }
            part[u] = t;
        }
        if (gain) gain[i] = g;
    }
    return OR_OK;
}
