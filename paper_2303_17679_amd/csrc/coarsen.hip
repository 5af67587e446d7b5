// Clustering pass of coarsening (paper Sec. 4.1: heavy-edge rating,
// contraction limit, cluster weight limit c_max; Sec. 11: deterministic
// clustering with sub-rounds, group-by target, ascending-weight prefix).
//
// GPU design.  A sub-round has three steps.
//  1. Rating.  Each candidate u aggregates r(u,C) over the clusters of its
//     neighbourhood in a hash table of its own.  Candidates are binned once
//     per level by B(u) = sum over incident nets (|e|-1), an upper bound on
//     their distinct neighbour clusters: groups of 8, 16 or 64 lanes with
//     LDS tables of 64 / 256 / 1024 entries (load <= 2/3), a whole block
//     with a 4096-entry LDS table, or a block with a table slice in global
//     memory.  A group walks the incident nets one at a time, the lanes over
//     the pins; a per-slot "last net" stamp (atomic exchange) lets exactly one
//     lane add w(e)/(|e|-1) per (net, cluster), which is the set semantics of
//     the rating formula.  The argmax (rating desc, tie hash asc, ID asc) is a
//     shuffle reduction.  The winning join adds c(u) to tsum[C] (integer
//     atomics: order independent), the paper's "sum up cluster weights during
//     the target-cluster calculation".
//  2. Approval.  A target whose whole group fits (160k (c(C) + tsum) <= c(V))
//     approves all joins.  The others go through a stable radix sort on
//     (C, c(u), u) and a prefix-sum test: the longest fitting prefix is
//     approved.
//  3. Apply: rep, cluster weights and the cluster count.
#include "prims.h"
#include "kernels.h"
#include "timing.h"

namespace hgp {

constexpr int NCLASS = 5;  // 0..2 wave groups, 3 block/LDS, 4 block/global
static const uint32_t CLASS_MAXB[4] = {42, 170, 682, 2730};

struct RateArgs {
    const uint32_t *pin_off, *pins, *inc_off, *inc;
    const int32_t *vwgt;
    const uint64_t *nscore;
    const uint32_t *rep;
    const int64_t *cw;
    const int64_t *tinfo;  // cluster weight of a valid target, TINFO_BAD otherwise
    uint32_t *ptarget;
    int64_t *tsum;
    uint64_t mseed;
    uint32_t level, r, S;
    int64_t cap_mult, W;
    bool dedup;  // false in the first sub-round: every cluster is a singleton
    const uint32_t *ncl;  // clusters after the previous sub-round
    uint32_t n_cur;       // vertices of the level
    const uint32_t *ovf;  // set: an earlier sub-round awaits the host (nullptr: none can)
    // community of every vertex (Sec. 4.3): u may join only a cluster whose
    // representative lies in its community; nullptr: no restriction
    const uint32_t *comm;
};

// The pass stops once the clustering has shrunk the level below n / 2.5
// (checked after every sub-round): the kernels of the remaining sub-rounds
// see it on the device and do nothing.
__device__ inline bool pass_cut(const uint32_t *ncl, uint32_t n) {
    return (uint64_t)5 * *ncl < (uint64_t)2 * n;
}

// A pass whose sub-rounds are all queued at once: the sorted approval of a
// sub-round runs in one workgroup, and one too large for it sets ovf to
// 1 + the sub-round, after which every later kernel of the pass does
// nothing until the host has finished that sub-round.  cut[r] keeps the
// pass-cut decision of sub-round r, taken before its joins change the
// cluster count.
__device__ inline bool ovf_set(const uint32_t *ovf) { return ovf && *ovf != 0; }
__device__ inline bool rate_skip(const RateArgs &a) { return ovf_set(a.ovf) || pass_cut(a.ncl, a.n_cur); }

// Larger than any cluster weight (< 2^31) while cap_mult * (c(u) + TINFO_BAD)
// stays far from overflow (cap_mult = limit_factor * k < 2^26).
constexpr int64_t TINFO_BAD = (int64_t)1 << 34;

// tinfo[C]: cw[C] if C may be joined in sub-round r, TINFO_BAD if C is itself
// a candidate singleton of the sub-round (no chains within a sub-round).
// Every vertex of the sub-round starts with no target.
// Block 0 also clears the slow-join count and records the pass-cut decision.
__global__ void k_target_info(const uint32_t *rep, const int64_t *cw, const int32_t *vwgt, uint32_t n,
                              uint64_t mseed, uint32_t level, uint32_t S, uint32_t r, int64_t *tinfo,
                              uint32_t *ptarget, const uint32_t *ncl, uint32_t *nslow, uint32_t *cut,
                              const uint32_t *ovf) {
    if (ovf_set(ovf)) return;
    const bool c = pass_cut(ncl, n);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *nslow = 0;
        cut[r] = c ? 1u : 0u;
    }
    if (c) return;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int64_t c = cw[v];
        const bool mine = tag_hash(mseed, 1, level, 0, v) % S == r;
        bool cand = rep[v] == v && c == (int64_t)vwgt[v] && mine;
        tinfo[v] = cand ? TINFO_BAD : c;
        if (mine) ptarget[v] = NONE;
    }
}

// (R1, C1) better than (R2, C2): larger rating, then smaller tie hash, then
// smaller ID.  The tie hash is computed only when the ratings are equal.
__device__ inline bool better_lazy(const RateArgs &a, uint64_t R1, uint32_t C1, uint64_t R2, uint32_t C2) {
    if (C2 == NONE) return C1 != NONE;
    if (C1 == NONE) return false;
    if (R1 != R2) return R1 > R2;
    uint64_t H1 = tag_hash(a.mseed, 2, a.level, 0, C1), H2 = tag_hash(a.mseed, 2, a.level, 0, C2);
    if (H1 != H2) return H1 < H2;
    return C1 < C2;
}

__device__ inline uint32_t slot_hash(uint32_t C, int log2cap) {
    return (uint32_t)(C * 2654435761u) >> (32 - log2cap);
}

// Validity of target cluster C for candidate u on the sub-round snapshot:
// within c_max and not a candidate singleton of the same sub-round.
__device__ inline bool valid_target(const RateArgs &a, uint32_t u, uint32_t C) {
    return C != u && a.cap_mult * ((int64_t)a.vwgt[u] + a.tinfo[C]) <= a.W && (!a.comm || a.comm[C] == a.comm[u]);
}

// Called by the publishing lanes only.  The sub-round's candidate list is
// its proposer list: k_target_info has set ptarget to NONE for every
// candidate, so no proposer is appended anywhere (a shared append counter
// costs one serialised device-scope atomic per wave).
__device__ inline void publish(const RateArgs &a, uint32_t u, uint32_t C) {
    if (C == NONE) return;
    a.ptarget[u] = C;
    atomic_add_i64(&a.tsum[C], (int64_t)a.vwgt[u]);
}

// Nets with at most LANE_NET pins are rated by a single lane: it loads the
// net's pins and their clusters at once and drops repeated clusters in
// registers, so every distinct (net, cluster) pair adds w(e)/(|e|-1) exactly
// once without any ordering between lanes.  Larger nets are processed by the
// whole group, one net at a time, with a per-slot "last net" stamp.
constexpr uint32_t LANE_NET = 16;

// LN (at most LANE_NET) bounds the net size of the lane path; a level whose
// nets have at most 8 pins uses LN = 8, so a lane carries half the registers
// and comparisons.
template <uint32_t LN = LANE_NET, class Insert>
__device__ inline void rate_small_net(const RateArgs &a, uint32_t u, uint32_t b, uint32_t sz, uint64_t sc,
                                      Insert &&insert) {
    uint32_t C[LN];
#pragma unroll
    for (uint32_t q = 0; q < LN; ++q) C[q] = q < sz ? a.pins[b + q] : NONE;
#pragma unroll
    for (uint32_t q = 0; q < LN; ++q)  // (first sub-round: every vertex is its own cluster)
        C[q] = (C[q] != NONE && C[q] != u) ? (a.dedup ? a.rep[C[q]] : C[q]) : NONE;
#pragma unroll
    for (uint32_t q = 0; q < LN; ++q) {
        bool fresh = C[q] != NONE;
#pragma unroll
        for (uint32_t r = 0; r < q; ++r) fresh = fresh && C[r] != C[q];
        if (fresh) insert(C[q], sc);
    }
}

// ---------------------------------------------------------------------------
// Groups of G lanes (G <= 64), one candidate per group, LDS table of CAP.
// Occupied slots are listed so that argmax and clearing touch only them.
// A large net adds its score once per cluster: a bit per slot marks the
// clusters it has reached (cleared before each large net).
// ---------------------------------------------------------------------------
// Workgroup sizes of the rating classes: the tables take about 27 KB (8
// lanes) and 54-58 KB (16, 64 lanes) of LDS per 256 threads, so smaller
// workgroups let more waves share a CU's LDS.
constexpr int RATE_NT8 = 128, RATE_NT = 64;
template <int G, int CAP, int LOG2CAP, uint32_t LN, int NT = BLOCK>
__global__ __launch_bounds__(NT) void k_rate_group(RateArgs a, const uint32_t *list, uint32_t count) {
    constexpr int GPB = NT / G;
    constexpr int MW = CAP / 64;  // mask words per group
    if (rate_skip(a)) return;
    __shared__ uint32_t keys[GPB][CAP];
    __shared__ unsigned long long seen[GPB][MW];
    __shared__ uint64_t R[GPB][CAP];
    using OccT = typename std::conditional<(CAP <= 256), uint8_t, uint16_t>::type;  // slot indices
    __shared__ OccT occ[GPB][CAP];
    __shared__ uint32_t nocc[GPB];
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int s = l; s < CAP; s += G) { keys[g][s] = NONE; R[g][s] = 0; }
    if (l == 0) nocc[g] = 0;
    wave_sync();
    // groups never synchronise with each other (each lives inside one wave),
    // so every group simply strides over the list.  The candidates' records
    // are fetched ahead (this kernel writes none of them): the ID two
    // candidates ahead, and the cluster state and incidence range of the
    // next, so those loads overlap the current candidate's gathers.
    // XCD x takes the x-th eighth of the list (the lists hold the vertices
    // in ascending order of classify block, i.e. about in vertex order), so
    // candidates that share nets share an L2
    const XcdSlice xs = xcd_slice(blockIdx.x, gridDim.x, count);
    const uint32_t stride = xs.nw * GPB, end = xs.hi;
    uint32_t idx = xs.lo + xs.wi * GPB + g;
    uint32_t pu = NONE, pj0 = 0, pj1 = 0;  // the next candidate's record
    int64_t pcw = 0;
    int32_t pvw = 0;
    uint32_t prep = NONE;
    auto fetch = [&](uint32_t v) {
        pu = v;
        if (v != NONE) {
            prep = a.rep[v];
            pcw = a.cw[v];
            pvw = a.vwgt[v];
            pj0 = a.inc_off[v];
            pj1 = a.inc_off[v + 1];
        }
    };
    fetch(idx < end ? list[idx] : NONE);
    uint32_t nid = idx + stride < end ? list[idx + stride] : NONE;  // the ID after that
    for (; idx < end; idx += stride) {
        const uint32_t u = pu, j0 = pj0, j1 = pj1;
        const int64_t cu = pvw;
        const bool active = prep == u && pcw == cu;  // not joined earlier
        const uint32_t after = nid;
        nid = idx + 2 * stride < end ? list[idx + 2 * stride] : NONE;
        fetch(after);
        if (!active) continue;  // uniform within the group
        auto insert = [&](uint32_t C, uint64_t sc) -> uint32_t {
            uint32_t slot = slot_hash(C, LOG2CAP);
            for (;;) {
                uint32_t k = keys[g][slot];
                if (k == C) break;
                if (k == NONE) {
                    uint32_t old = atomicCAS(&keys[g][slot], NONE, C);
                    if (old == NONE) {
                        occ[g][atomicAdd(&nocc[g], 1u)] = (OccT)slot;
                        break;
                    }
                    if (old == C) break;
                }
                slot = (slot + 1) & (CAP - 1);
            }
            return slot;
        };
        // phase 1: small nets, one lane each
        bool big = false;
        for (uint32_t j = j0 + l; j < j1; j += G) {
            uint32_t e = a.inc[j];
            uint32_t b = a.pin_off[e], sz = a.pin_off[e + 1] - b;
            if (sz > LN) { big = true; continue; }
            if (sz < 2) continue;
            rate_small_net<LN>(a, u, b, sz, a.nscore[e], [&](uint32_t C, uint64_t sc) {
                uint32_t slot = insert(C, sc);
                atomicAdd((unsigned long long *)&R[g][slot], (unsigned long long)sc);
            });
        }
        // phase 2: large nets, the whole group on one net at a time
        uint64_t bigmask = __ballot(big);
        const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << ((__lane_id() / G) * G));
        wave_sync();
        if (bigmask & gmask) {
            for (uint32_t j = j0; j < j1; ++j) {
                uint32_t e = a.inc[j];
                uint32_t b = a.pin_off[e], sz = a.pin_off[e + 1] - b;
                if (sz <= LN) continue;
                uint64_t sc = a.nscore[e];
                if (a.dedup) {
                    for (int w = l; w < MW; w += G) seen[g][w] = 0ull;
                    wave_sync();
                }
                for (uint32_t q = l; q < sz; q += G) {
                    uint32_t v = a.pins[b + q];
                    if (v == u) continue;
                    const uint32_t slot = insert(a.dedup ? a.rep[v] : v, sc);
                    bool first = true;
                    if (a.dedup) {
                        const unsigned long long bit = 1ull << (slot & 63);
                        first = (atomicOr(&seen[g][slot >> 6], bit) & bit) == 0ull;
                    }
                    if (first) atomicAdd((unsigned long long *)&R[g][slot], (unsigned long long)sc);
                }
                wave_sync();
            }
        }
        wave_sync();
        const uint32_t no = nocc[g];
        uint64_t bR = 0;
        uint32_t bC = NONE;
        // four slots per lane at a time so that their tinfo loads overlap
        for (uint32_t i0 = 0; i0 < no; i0 += 4 * G) {
            uint32_t Cs[4];
            uint64_t Rs[4];
            int64_t Ts[4];
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                uint32_t i = i0 + k4 * G + l;
                Cs[k4] = NONE;
                Rs[k4] = 0;
                if (i < no) {
                    uint32_t slot = occ[g][i];
                    Cs[k4] = keys[g][slot];
                    Rs[k4] = R[g][slot];
                    keys[g][slot] = NONE;  // leave the table clean for the next candidate
                    R[g][slot] = 0;
                }
            }
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) Ts[k4] = Cs[k4] != NONE ? a.tinfo[Cs[k4]] : TINFO_BAD;
            if (a.comm) {  // a cluster of another community is no target (Sec. 4.3)
                const uint32_t cmu = a.comm[u];
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4)
                    if (Cs[k4] != NONE && a.comm[Cs[k4]] != cmu) Ts[k4] = TINFO_BAD;
            }
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                bool ok = Cs[k4] != NONE && Cs[k4] != u && a.cap_mult * (cu + Ts[k4]) <= a.W;
                if (ok && better_lazy(a, Rs[k4], Cs[k4], bR, bC)) { bR = Rs[k4]; bC = Cs[k4]; }
            }
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            uint64_t oR = __shfl_xor(bR, o, 64);
            uint32_t oC = __shfl_xor(bC, o, 64);
            if (better_lazy(a, oR, oC, bR, bC)) { bR = oR; bC = oC; }
        }
        wave_sync();
        if (l == 0) {
            publish(a, u, bC);
            nocc[g] = 0;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// One candidate per block; table of LCAP slots in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_rate_block(RateArgs a, const uint32_t *list, uint32_t count) {
    constexpr int LCAP = 4096, LLOG = 12;
    if (rate_skip(a)) return;
    __shared__ uint32_t keys[LCAP];
    __shared__ uint32_t stamp[LCAP];
    __shared__ uint64_t R[LCAP];
    __shared__ uint64_t redR[BLOCK / WAVE];
    __shared__ uint32_t redC[BLOCK / WAVE];
    const XcdSlice xs = xcd_slice(blockIdx.x, gridDim.x, count);
    for (uint32_t idx = xs.lo + xs.wi; idx < xs.hi; idx += xs.nw) {
        uint32_t u = list[idx];
        if (!(a.rep[u] == u && a.cw[u] == (int64_t)a.vwgt[u])) continue;  // uniform per block
        for (uint32_t s = threadIdx.x; s < LCAP; s += BLOCK) { keys[s] = NONE; stamp[s] = NONE; R[s] = 0; }
        __syncthreads();
        uint32_t j0 = a.inc_off[u], j1 = a.inc_off[u + 1];
        auto insert = [&](uint32_t C) -> uint32_t {
            uint32_t slot = slot_hash(C, LLOG);
            for (;;) {
                uint32_t k = keys[slot];
                if (k == C) break;
                if (k == NONE) {
                    uint32_t old = atomicCAS(&keys[slot], NONE, C);
                    if (old == NONE || old == C) break;
                }
                slot = (slot + 1) & (LCAP - 1);
            }
            return slot;
        };
        // phase 1: small nets, one thread each
        int big = 0;
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += BLOCK) {
            uint32_t e = a.inc[j];
            uint32_t b = a.pin_off[e], sz = a.pin_off[e + 1] - b;
            if (sz > LANE_NET) { big = 1; continue; }
            if (sz < 2) continue;
            rate_small_net(a, u, b, sz, a.nscore[e], [&](uint32_t C, uint64_t sc) {
                uint32_t slot = insert(C);
                atomicAdd((unsigned long long *)&R[slot], (unsigned long long)sc);
            });
        }
        // phase 2: large nets, the whole block on one net at a time
        const int anybig = __syncthreads_or(big);
        __syncthreads();  // phase-1 table updates complete before anyone reads the table
        if (anybig) {
            for (uint32_t j = j0; j < j1; ++j) {
                uint32_t e = a.inc[j];
                uint32_t b = a.pin_off[e], sz = a.pin_off[e + 1] - b;
                if (sz <= LANE_NET) continue;
                uint64_t sc = a.nscore[e];
                for (uint32_t q = threadIdx.x; q < sz; q += BLOCK) {
                    uint32_t v = a.pins[b + q];
                    if (v == u) continue;
                    uint32_t slot = insert(a.rep[v]);
                    if (!a.dedup || atomicExch(&stamp[slot], e) != e)
                        atomicAdd((unsigned long long *)&R[slot], (unsigned long long)sc);
                }
                __syncthreads();
            }
        }
        uint64_t bR = 0;
        uint32_t bC = NONE;
        for (uint32_t s = threadIdx.x; s < LCAP; s += BLOCK) {
            const uint32_t C = keys[s];
            if (C == NONE) continue;
            if (valid_target(a, u, C) && better_lazy(a, R[s], C, bR, bC)) { bR = R[s]; bC = C; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            uint64_t oR = __shfl_xor(bR, o, 64);
            uint32_t oC = __shfl_xor(bC, o, 64);
            if (better_lazy(a, oR, oC, bR, bC)) { bR = oR; bC = oC; }
        }
        unsigned w = threadIdx.x / WAVE;
        if (__lane_id() == 0) { redR[w] = bR; redC[w] = bC; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < BLOCK / WAVE; ++q)
                if (better_lazy(a, redR[q], redC[q], bR, bC)) { bR = redR[q]; bC = redC[q]; }
            publish(a, u, bC);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Hub rating: candidates whose cluster bound D exceeds the LDS tables.  Such a
// vertex can have ~1e5 incident nets, so its rating is spread over many
// workgroups that share one global table per candidate (a "job"):
//   k_hub_info    - (u, incidence range, D) of every listed candidate;
//   k_hub_insert  - one workgroup per item (up to HUB_CHUNK incident nets of
//                   one job): nets of <= LANE_NET pins one thread each
//                   (clusters deduplicated in registers), nets of up to
//                   HUB_BIG pins by the whole workgroup through an LDS set
//                   (each cluster of the net once), larger nets skipped;
//   k_hub_huge    - one workgroup per job: its nets of more than HUB_BIG pins,
//                   one at a time, deduplicated by a per-slot net stamp (no
//                   other net of the job is in flight then);
//   k_hub_argmax  - one workgroup per slice of ARG_SLICE slots of a job's
//                   table: the best target of the slice (used slots are
//                   reset);
//   k_hub_pick    - a wave per job: the best of its slices, published.
// Tables start clean (the host clears the region once per pass) and are left
// clean.  No list of used slots is kept: a shared counter per job would be
// one address that every insert of the job hits.
// ---------------------------------------------------------------------------
constexpr uint32_t HUB_CHUNK = BLOCK;
constexpr uint32_t HUB_BIG = 2048;
constexpr uint32_t HUB_SET = 4096;  // power of two >= 2 * HUB_BIG

struct HubJob {
    uint32_t u, lg;  // candidate, log2 of its table capacity
    uint32_t j0, j1; // its incidence range
    uint64_t off;    // first entry of its table in the region
    uint32_t pbase, nslice;  // its argmax slices: partial results [pbase, pbase + nslice)
};
constexpr uint32_t ARG_SLICE = 4096;  // table slots per argmax workgroup
constexpr uint32_t HUB_WORK = 8192;   // about this many pins per insert item
constexpr uint32_t HUB_MIN_NETS = 32; // but at least this many incident nets
struct HubItem {
    uint32_t job, j0, j1, pad;
};

__global__ __launch_bounds__(BLOCK) void k_hub_info(RateArgs a, const uint32_t *list, uint32_t count,
                                                    const uint32_t *bound, uint32_t n_cur, uint4 *info) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        const uint32_t u = list[i];
        const bool active = a.rep[u] == u && a.cw[u] == (int64_t)a.vwgt[u] && !rate_skip(a);
        const uint32_t D = bound[u] < n_cur - 1 ? bound[u] : n_cur - 1;
        info[i] = make_uint4(u, a.inc_off[u], a.inc_off[u + 1], active ? D : NONE);
    }
}

// Insert cluster C of job J into its table; returns the slot.  Within a
// kernel a key only ever goes from NONE to a cluster, so the probe may read
// it through this XCD's L2 (workgroup scope) even if another XCD has just
// claimed the slot: a stale NONE only leads to the CAS, which is device-wide
// and returns the key actually there, and a key once read never changes.
__device__ inline uint32_t hub_slot(uint32_t *keys, const HubJob &J, uint32_t C) {
    const uint32_t mask = (1u << J.lg) - 1u;
    uint32_t *kt = keys + J.off;
    uint32_t slot = slot_hash(C, (int)J.lg);
    for (;;) {
        const uint32_t k = __hip_atomic_load(&kt[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == C) return slot;
        if (k == NONE) {
            const uint32_t old = atomicCAS(&kt[slot], NONE, C);
            if (old == NONE || old == C) return slot;
        }
        slot = (slot + 1) & mask;
    }
}

// Nets of more than LANE_NET pins are taken in windows of whole nets with at
// most HUB_WIN pins together; the workgroup spreads each window's pins over
// all its threads, and a (net, cluster) set in LDS lets the first pin of a
// net in a cluster claim the pair.
constexpr uint32_t HUB_WIN = 2048;
__global__ __launch_bounds__(BLOCK) void k_hub_insert(RateArgs a, const HubJob *jobs, const HubItem *items,
                                                      uint32_t nitems, uint32_t *keys, uint64_t *R) {
    __shared__ unsigned long long set[HUB_SET];  // (net index in the item << 32) | cluster
    __shared__ uint16_t setocc[HUB_SET];
    __shared__ uint32_t nset;
    __shared__ uint32_t bstart[HUB_CHUNK + 1];  // first flattened pin of each listed net
    __shared__ uint32_t bpin[HUB_CHUNK];        // its first pin in the pin array
    __shared__ uint64_t bsc[HUB_CHUNK];         // its score
    __shared__ uint32_t wsum[BLOCK / WAVE];
    constexpr unsigned long long EMPTY = ~0ull;
    for (uint32_t q = threadIdx.x; q < HUB_SET; q += BLOCK) set[q] = EMPTY;
    if (threadIdx.x == 0) nset = 0;
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const HubItem I = items[it];
        const HubJob J = jobs[I.job];
        const uint32_t u = J.u;
        __syncthreads();
        // small nets: one thread each; the others are listed in incidence order
        const uint32_t j = I.j0 + threadIdx.x;
        uint32_t bsz = 0, e = 0, b = 0;
        if (j < I.j1) {
            e = a.inc[j];
            b = a.pin_off[e];
            const uint32_t sz = a.pin_off[e + 1] - b;
            if (sz >= 2 && sz <= LANE_NET) {
                rate_small_net(a, u, b, sz, a.nscore[e], [&](uint32_t C, uint64_t sc) {
                    const uint32_t slot = hub_slot(keys, J, C);
                    atomicAdd((unsigned long long *)&R[J.off + slot], (unsigned long long)sc);
                });
            } else if (sz > LANE_NET && sz <= HUB_BIG) {
                bsz = sz;
            }
        }
        uint32_t tot_n, tot_p;
        const uint32_t rank = block_incl_scan<uint32_t>(bsz ? 1u : 0u, wsum, &tot_n) - (bsz ? 1u : 0u);
        const uint32_t pre = block_incl_scan<uint32_t>(bsz, wsum, &tot_p) - bsz;
        if (bsz) {
            bstart[rank] = pre;
            bpin[rank] = b;
            bsc[rank] = a.nscore[e];
        }
        if (threadIdx.x == 0) bstart[tot_n] = tot_p;
        __syncthreads();
        const uint32_t nb = tot_n;
        for (uint32_t w0 = 0; w0 < nb;) {
            // the window: nets w0 .. w1-1, at least one, at most HUB_WIN pins
            uint32_t lo = w0 + 1, hi = nb;  // largest w1 with bstart[w1] - bstart[w0] <= HUB_WIN
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (bstart[mid] - bstart[w0] <= HUB_WIN) lo = mid; else hi = mid - 1;
            }
            const uint32_t w1 = lo;
            for (uint32_t x = bstart[w0] + threadIdx.x; x < bstart[w1]; x += BLOCK) {
                uint32_t tl = w0, th = w1 - 1;  // net of flattened pin x
                while (tl < th) {
                    const uint32_t mid = (tl + th + 1) >> 1;
                    if (bstart[mid] <= x) tl = mid; else th = mid - 1;
                }
                const uint32_t v = a.pins[bpin[tl] + (x - bstart[tl])];
                if (v == u) continue;
                const uint32_t C = a.rep[v];
                bool fresh = true;
                if (a.dedup) {  // first pin of the net in cluster C claims the pair
                    const unsigned long long key = ((unsigned long long)tl << 32) | C;
                    uint32_t h = slot_hash(C ^ (tl * 0x9E3779B9u), 12);
                    for (;;) {
                        const unsigned long long k = set[h];
                        if (k == key) { fresh = false; break; }
                        if (k == EMPTY) {
                            const unsigned long long old = atomicCAS(&set[h], EMPTY, key);
                            if (old == EMPTY) { setocc[atomicAdd(&nset, 1u)] = (uint16_t)h; break; }
                            if (old == key) { fresh = false; break; }
                        }
                        h = (h + 1) & (HUB_SET - 1);
                    }
                }
                if (fresh) {
                    const uint32_t slot = hub_slot(keys, J, C);
                    atomicAdd((unsigned long long *)&R[J.off + slot], (unsigned long long)bsc[tl]);
                }
            }
            __syncthreads();
            if (a.dedup) {
                const uint32_t ns = nset;
                for (uint32_t x = threadIdx.x; x < ns; x += BLOCK) set[setocc[x]] = EMPTY;
                __syncthreads();
                if (threadIdx.x == 0) nset = 0;
                __syncthreads();
            }
            w0 = w1;
        }
    }
}

// ---------------------------------------------------------------------------
// Hub jobs of moderate bound D (and levels without nets of more than HUB_BIG
// pins): the rating is aggregated in LDS instead of a global table, one
// workgroup per job with a table of LHUB_CAP slots.  The kernel can also
// split the clusters into P partitions by a hash (a workgroup per (job,
// partition), each reading all of the job's pins), but P = 1 is used: with
// D <= LHUB_PART the table cannot fill (D bounds the distinct clusters), and
// splitting costs more pin reads than the global table it replaces.  A table
// that does fill marks the job, which is then rated on the global path.
// ---------------------------------------------------------------------------
constexpr int LHUB_THREADS = 512;
constexpr uint32_t LHUB_CAP = 8192, LHUB_LG = 13;
constexpr uint32_t LHUB_PART = 5461;  // clusters per partition at most (load 2/3)
constexpr uint32_t LHUB_MAXP = 1;

__device__ inline uint32_t lhub_part(uint32_t C, uint32_t P) {
    return (uint32_t)(((uint64_t)(C * 0x85EBCA6Bu) * P) >> 32);
}

__global__ __launch_bounds__(LHUB_THREADS) void k_hub_lds(RateArgs a, const HubJob *jobs, const HubItem *litems,
                                                          uint32_t nl, uint64_t *partR, uint32_t *partC,
                                                          uint32_t *ovf_flag, uint32_t *ovf_list, uint32_t *ovf_cnt) {
    __shared__ uint32_t tkey[LHUB_CAP];
    __shared__ unsigned long long tR[LHUB_CAP];
    __shared__ unsigned long long set[HUB_SET];  // (net index in the chunk << 32) | cluster
    __shared__ uint16_t setocc[HUB_SET];
    __shared__ uint32_t nset, ovf;
    __shared__ uint32_t bstart[LHUB_THREADS + 1];
    __shared__ uint32_t bpin[LHUB_THREADS];
    __shared__ uint64_t bsc[LHUB_THREADS];
    __shared__ uint32_t wsum[LHUB_THREADS / WAVE];
    __shared__ uint64_t redR[LHUB_THREADS / WAVE];
    __shared__ uint32_t redC[LHUB_THREADS / WAVE];
    constexpr unsigned long long EMPTY = ~0ull;
    const uint32_t tid = threadIdx.x;
    for (uint32_t q = tid; q < HUB_SET; q += LHUB_THREADS) set[q] = EMPTY;
    if (tid == 0) nset = 0;
    for (uint32_t it = blockIdx.x; it < nl; it += gridDim.x) {
        const HubItem I = litems[it];
        const HubJob J = jobs[I.job];
        const uint32_t u = J.u, P = J.lg, part = I.j0;
        __syncthreads();
        for (uint32_t q = tid; q < LHUB_CAP; q += LHUB_THREADS) { tkey[q] = NONE; tR[q] = 0; }
        if (tid == 0) ovf = 0;
        __syncthreads();
        auto tins = [&](uint32_t C, uint64_t sc) {
            uint32_t slot = slot_hash(C, LHUB_LG);
            for (uint32_t probe = 0; probe < LHUB_CAP; ++probe) {
                const uint32_t k = tkey[slot];
                if (k == C) { atomicAdd(&tR[slot], (unsigned long long)sc); return; }
                if (k == NONE) {
                    const uint32_t old = atomicCAS(&tkey[slot], NONE, C);
                    if (old == NONE || old == C) { atomicAdd(&tR[slot], (unsigned long long)sc); return; }
                }
                slot = (slot + 1) & (LHUB_CAP - 1);
            }
            ovf = 1;  // the table is full
        };
        for (uint32_t c0 = J.j0; c0 < J.j1; c0 += LHUB_THREADS) {
            // nets of <= LANE_NET pins: one thread each; the others are listed
            const uint32_t j = c0 + tid;
            uint32_t bsz = 0, e = 0, b = 0;
            if (j < J.j1) {
                e = a.inc[j];
                b = a.pin_off[e];
                const uint32_t sz = a.pin_off[e + 1] - b;
                if (sz >= 2 && sz <= LANE_NET) {
                    rate_small_net(a, u, b, sz, a.nscore[e], [&](uint32_t C, uint64_t sc) {
                        if (lhub_part(C, P) == part) tins(C, sc);
                    });
                } else if (sz > LANE_NET) {
                    bsz = sz;  // <= HUB_BIG on the levels that take this path
                }
            }
            uint32_t tot_n, tot_p;
            const uint32_t rank =
                block_incl_scan_n<uint32_t, LHUB_THREADS>(bsz ? 1u : 0u, wsum, &tot_n) - (bsz ? 1u : 0u);
            const uint32_t pre = block_incl_scan_n<uint32_t, LHUB_THREADS>(bsz, wsum, &tot_p) - bsz;
            if (bsz) {
                bstart[rank] = pre;
                bpin[rank] = b;
                bsc[rank] = a.nscore[e];
            }
            if (tid == 0) bstart[tot_n] = tot_p;
            __syncthreads();
            const uint32_t nb = tot_n;
            for (uint32_t w0 = 0; w0 < nb;) {
                uint32_t lo = w0 + 1, hi = nb;  // window: nets w0 .. w1-1 of at most HUB_WIN pins
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (bstart[mid] - bstart[w0] <= HUB_WIN) lo = mid; else hi = mid - 1;
                }
                const uint32_t w1 = lo;
                for (uint32_t x = bstart[w0] + tid; x < bstart[w1]; x += LHUB_THREADS) {
                    uint32_t tl = w0, th = w1 - 1;
                    while (tl < th) {
                        const uint32_t mid = (tl + th + 1) >> 1;
                        if (bstart[mid] <= x) tl = mid; else th = mid - 1;
                    }
                    const uint32_t v = a.pins[bpin[tl] + (x - bstart[tl])];
                    if (v == u) continue;
                    const uint32_t C = a.rep[v];
                    if (lhub_part(C, P) != part) continue;
                    bool fresh = true;
                    if (a.dedup) {
                        const unsigned long long key = ((unsigned long long)tl << 32) | C;
                        uint32_t h = slot_hash(C ^ (tl * 0x9E3779B9u), 12);
                        for (;;) {
                            const unsigned long long k = set[h];
                            if (k == key) { fresh = false; break; }
                            if (k == EMPTY) {
                                const unsigned long long old = atomicCAS(&set[h], EMPTY, key);
                                if (old == EMPTY) { setocc[atomicAdd(&nset, 1u)] = (uint16_t)h; break; }
                                if (old == key) { fresh = false; break; }
                            }
                            h = (h + 1) & (HUB_SET - 1);
                        }
                    }
                    if (fresh) tins(C, bsc[tl]);
                }
                __syncthreads();
                if (a.dedup) {
                    const uint32_t ns = nset;
                    for (uint32_t x = tid; x < ns; x += LHUB_THREADS) set[setocc[x]] = EMPTY;
                    __syncthreads();
                    if (tid == 0) nset = 0;
                    __syncthreads();
                }
                w0 = w1;
            }
            __syncthreads();  // bstart / bpin / bsc are rewritten by the next chunk
        }
        __syncthreads();
        uint64_t bR = 0;
        uint32_t bC = NONE;
        if (!ovf) {
            for (uint32_t q = tid; q < LHUB_CAP; q += LHUB_THREADS) {
                const uint32_t C = tkey[q];
                if (C == NONE) continue;
                const uint64_t rc = tR[q];
                if (valid_target(a, u, C) && better_lazy(a, rc, C, bR, bC)) { bR = rc; bC = C; }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t oR = __shfl_xor(bR, o, 64);
            const uint32_t oC = __shfl_xor(bC, o, 64);
            if (better_lazy(a, oR, oC, bR, bC)) { bR = oR; bC = oC; }
        }
        const unsigned w = tid / WAVE;
        if (__lane_id() == 0) { redR[w] = bR; redC[w] = bC; }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < LHUB_THREADS / WAVE; ++q)
                if (better_lazy(a, redR[q], redC[q], bR, bC)) { bR = redR[q]; bC = redC[q]; }
            partR[J.pbase + part] = bR;
            partC[J.pbase + part] = bC;
            if (ovf && atomicExch(&ovf_flag[I.job], 1u) == 0u) ovf_list[atomicAdd(ovf_cnt, 1u)] = I.job;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_hub_huge(RateArgs a, const HubJob *jobs, uint32_t njobs, uint32_t *keys,
                                                    uint32_t *stamp, uint64_t *R) {
    for (uint32_t jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
        const HubJob J = jobs[jb];
        for (uint32_t j = J.j0; j < J.j1; ++j) {
            const uint32_t e = a.inc[j];
            const uint32_t b = a.pin_off[e], sz = a.pin_off[e + 1] - b;
            if (sz <= HUB_BIG) continue;  // uniform per workgroup
            const uint64_t sc = a.nscore[e];
            for (uint32_t x = threadIdx.x; x < sz; x += BLOCK) {
                const uint32_t v = a.pins[b + x];
                if (v == J.u) continue;
                const uint32_t slot = hub_slot(keys, J, a.rep[v]);
                if (!a.dedup || atomicExch(&stamp[J.off + slot], e) != e)
                    atomicAdd((unsigned long long *)&R[J.off + slot], (unsigned long long)sc);
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_hub_argmax(RateArgs a, const HubJob *jobs, const HubItem *aitems,
                                                      uint32_t naitems, uint32_t *keys, uint32_t *stamp, uint64_t *R,
                                                      uint64_t *partR, uint32_t *partC) {
    __shared__ uint64_t redR[BLOCK / WAVE];
    __shared__ uint32_t redC[BLOCK / WAVE];
    for (uint32_t it = blockIdx.x; it < naitems; it += gridDim.x) {
        const HubItem I = aitems[it];
        const HubJob J = jobs[I.job];
        const uint32_t u = J.u;
        const uint32_t cap = 1u << J.lg;
        const uint32_t i0 = I.j0 * ARG_SLICE, i1 = cap < i0 + ARG_SLICE ? cap : i0 + ARG_SLICE;
        uint64_t bR = 0;
        uint32_t bC = NONE;
        for (uint32_t i = i0 + threadIdx.x; i < i1; i += BLOCK) {
            const uint64_t s = J.off + i;
            // (the inserts finished in an earlier kernel: plain reads)
            const uint32_t C = keys[s];
            if (C == NONE) continue;
            const uint64_t rc = R[s];
            keys[s] = NONE;
            stamp[s] = NONE;
            R[s] = 0;
            if (valid_target(a, u, C) && better_lazy(a, rc, C, bR, bC)) { bR = rc; bC = C; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t oR = __shfl_xor(bR, o, 64);
            const uint32_t oC = __shfl_xor(bC, o, 64);
            if (better_lazy(a, oR, oC, bR, bC)) { bR = oR; bC = oC; }
        }
        const unsigned w = threadIdx.x / WAVE;
        if (__lane_id() == 0) { redR[w] = bR; redC[w] = bC; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < BLOCK / WAVE; ++q)
                if (better_lazy(a, redR[q], redC[q], bR, bC)) { bR = redR[q]; bC = redC[q]; }
            partR[J.pbase + I.j0] = bR;
            partC[J.pbase + I.j0] = bC;
        }
        __syncthreads();
    }
}

// skip (may be null): jobs whose LDS table filled up (rated again later)
__global__ __launch_bounds__(BLOCK) void k_hub_pick(RateArgs a, const HubJob *jobs, uint32_t njobs,
                                                    const uint64_t *partR, const uint32_t *partC,
                                                    const uint32_t *skip) {
    const uint32_t wid = (blockIdx.x * BLOCK + threadIdx.x) / WAVE, nw = gridDim.x * BLOCK / WAVE;
    for (uint32_t jb = wid; jb < njobs; jb += nw) {
        if (skip && skip[jb]) continue;  // uniform per wave
        const HubJob J = jobs[jb];
        uint64_t bR = 0;
        uint32_t bC = NONE;
        for (uint32_t q = __lane_id(); q < J.nslice; q += WAVE) {
            const uint64_t r = partR[J.pbase + q];
            const uint32_t c = partC[J.pbase + q];
            if (better_lazy(a, r, c, bR, bC)) { bR = r; bC = c; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t oR = __shfl_xor(bR, o, 64);
            const uint32_t oC = __shfl_xor(bC, o, 64);
            if (better_lazy(a, oR, oC, bR, bC)) { bR = oR; bC = oC; }
        }
        if (__lane_id() == 0) publish(a, J.u, bC);
    }
}

// ---------------------------------------------------------------------------
// Measurement only: compulsory bytes of one rating launch -- every distinct
// array element the launch must read or write, counted once (candidate data,
// incidence lists, the offsets / score / pins of every distinct net touched,
// the cluster of every distinct pin vertex, the target info of every distinct
// cluster, the target written).  Never runs in a timed step.
// ---------------------------------------------------------------------------
struct ListVertex {
    const uint32_t *list;
    __device__ uint32_t operator()(uint32_t i) const { return list[i]; }
};
struct JobVertex {
    const HubJob *jobs;
    __device__ uint32_t operator()(uint32_t i) const { return jobs[i].u; }
};
template <class Get>
__global__ __launch_bounds__(BLOCK) void k_account_rate(RateArgs a, Get get, uint32_t count,
                                                        uint32_t *nmark, uint32_t *vmark, uint32_t *cmark,
                                                        uint32_t stamp, unsigned long long *acc) {
    __shared__ unsigned long long red[BLOCK / WAVE];
    if (rate_skip(a)) return;
    unsigned long long bytes = 0;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += gridDim.x * blockDim.x) {
        const uint32_t u = get(idx);
        bytes += 4 + 4 + 8 + 4;  // list entry, rep[u], cw[u], vwgt[u]
        if (!(a.rep[u] == u && a.cw[u] == (int64_t)a.vwgt[u])) continue;
        const uint32_t j0 = a.inc_off[u], j1 = a.inc_off[u + 1];
        bytes += 4 + 4ull * (j1 - j0) + 4;  // inc_off, incidence list, target
        for (uint32_t j = j0; j < j1; ++j) {
            uint32_t e = a.inc[j];
            uint32_t b = a.pin_off[e], sz = a.pin_off[e + 1] - b;
            bool first = atomicExch(&nmark[e], stamp) != stamp;
            if (sz < 2) { if (first) bytes += 4; continue; }
            if (first) bytes += 4 + 8 + 4ull * sz;  // pin offset, score, pins
            for (uint32_t q = 0; q < sz; ++q) {
                uint32_t v = a.pins[b + q];
                if (v == u) continue;
                if (atomicExch(&vmark[v], stamp) != stamp) bytes += 4;  // rep[v]
                uint32_t C = a.rep[v];
                if (atomicExch(&cmark[C], stamp) != stamp) bytes += 8;  // tinfo[C]
            }
        }
    }
    bytes = wave_sum(bytes);
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = bytes;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
        atomicAdd(acc, t);
    }
}

// ---------------------------------------------------------------------------
// Per-level preparation
// ---------------------------------------------------------------------------
__global__ void k_net_score(const uint32_t *pin_off, const int32_t *nwgt, uint32_t m, uint64_t *nscore) {
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
        uint32_t sz = pin_off[e + 1] - pin_off[e];
        nscore[e] = sz >= 2 ? ((uint64_t)(uint32_t)nwgt[e] << 32) / (uint64_t)(sz - 1) : 0;
    }
}

__device__ inline int rate_class(uint64_t B) {
    if (B == 0) return -1;
    if (B <= 42) return 0;
    if (B <= 170) return 1;
    if (B <= 682) return 2;
    if (B <= 2730) return 3;
    return 4;
}

// Largest net size of the level, by the first NETMAX_BLOCKS blocks only: one
// device-scope atomic per block (atomics on one address are serialised).
constexpr uint32_t NETMAX_BLOCKS = 256;
__device__ inline void net_size_max(const uint32_t *pin_off, uint32_t m, uint32_t *maxsz) {
    if (blockIdx.x >= NETMAX_BLOCKS) return;
    __shared__ uint32_t red[BLOCK / WAVE];
    const uint32_t nb = gridDim.x < NETMAX_BLOCKS ? gridDim.x : NETMAX_BLOCKS;
    uint32_t mx = 0;
    for (uint32_t e = blockIdx.x * BLOCK + threadIdx.x; e < m; e += nb * BLOCK) {
        const uint32_t sz = pin_off[e + 1] - pin_off[e];
        mx = sz > mx ? sz : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BLOCK / WAVE; ++q) mx = red[q] > mx ? red[q] : mx;
        if (mx) atomicMax(maxsz, mx);
    }
}

// B(u) = sum over incident nets of at least two pins of (|e| - 1), a bound
// on the clusters a rating of u can touch.  Thread per vertex; a vertex of
// more than 32 incident nets is summed by its whole wave.
// Vertices of more than VB_HUGE nets are listed (huge, count in *nhuge) and
// summed by k_vertex_b_huge, a workgroup each, so that no wave walks a hub's
// incidence list alone.
constexpr uint32_t VB_HUGE = 8192;
__global__ __launch_bounds__(BLOCK) void k_vertex_b(const uint32_t *pin_off, const uint32_t *inc_off,
                                                    const uint32_t *inc, uint32_t n, uint32_t m, uint32_t *bound,
                                                    uint32_t *maxsz, uint32_t *huge, uint32_t *nhuge) {
    // largest net size of the level (decides whether the hub path needs its
    // huge-net kernel)
    net_size_max(pin_off, m, maxsz);
    for (uint32_t u0 = blockIdx.x * BLOCK; u0 < n; u0 += gridDim.x * BLOCK) {
        const uint32_t u = u0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (u < n) { j0 = inc_off[u]; j1 = inc_off[u + 1]; }
        const bool heavy = j1 - j0 > 32;
        uint64_t b = 0;
        if (!heavy)  // eight nets at a time: all incidence loads, then all offset loads
            for (uint32_t j = j0; j < j1; j += 8) {
                uint32_t e[8];
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) e[q] = j + q < j1 ? inc[j + q] : NONE;
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) {
                    if (e[q] == NONE) continue;
                    const uint32_t sz = pin_off[e[q] + 1] - pin_off[e[q]];
                    if (sz >= 2) b += sz - 1;
                }
            }
        const bool is_huge = heavy && j1 - j0 > VB_HUGE;
        const uint32_t at = warp_agg_append(nhuge, is_huge);
        if (is_huge) huge[at] = u;
        uint64_t hm = __ballot(heavy && !is_huge);
        while (hm) {  // the wave sums each heavy vertex together
            const int h = __ffsll((long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t hj0 = __shfl(j0, h, 64), hj1 = __shfl(j1, h, 64);
            uint64_t t = 0;
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) {
                const uint32_t e = inc[j];
                const uint32_t sz = pin_off[e + 1] - pin_off[e];
                if (sz >= 2) t += sz - 1;
            }
            t = wave_sum(t);
            if ((int)__lane_id() == h) b = t;
        }
        if (u < n && !is_huge) bound[u] = b > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)b;
    }
}

constexpr int VB_HUGE_THREADS = 1024;
__global__ __launch_bounds__(VB_HUGE_THREADS) void k_vertex_b_huge(const uint32_t *pin_off, const uint32_t *inc_off,
                                                                   const uint32_t *inc, const uint32_t *huge,
                                                                   const uint32_t *nhuge, uint32_t *bound) {
    __shared__ uint64_t red[VB_HUGE_THREADS / WAVE];
    const uint32_t cnt = *nhuge;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {  // uniform per block
        const uint32_t u = huge[i], j1 = inc_off[u + 1];
        uint64_t t = 0;
        for (uint32_t j = inc_off[u] + threadIdx.x; j < j1; j += VB_HUGE_THREADS) {
            const uint32_t e = inc[j];
            const uint32_t sz = pin_off[e + 1] - pin_off[e];
            if (sz >= 2) t += sz - 1;
        }
        t = wave_sum(t);
        if (__lane_id() == 0) red[threadIdx.x / WAVE] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < VB_HUGE_THREADS / WAVE; ++q) t += red[q];
            bound[u] = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
        }
        __syncthreads();
    }
}

// The same bound with a wave per vertex, for levels whose average degree is
// high (coarse levels): every vertex is summed by all 64 lanes at once.
__global__ __launch_bounds__(BLOCK) void k_vertex_b_wave(const uint32_t *pin_off, const uint32_t *inc_off,
                                                         const uint32_t *inc, uint32_t n, uint32_t m,
                                                         uint32_t *bound, uint32_t *maxsz, uint32_t *huge,
                                                         uint32_t *nhuge) {
    net_size_max(pin_off, m, maxsz);
    const uint32_t wid = (blockIdx.x * BLOCK + threadIdx.x) / WAVE, nw = gridDim.x * BLOCK / WAVE;
    for (uint32_t u = wid; u < n; u += nw) {
        const uint32_t j0 = inc_off[u], j1 = inc_off[u + 1];
        if (j1 - j0 > VB_HUGE) {  // uniform per wave
            if (__lane_id() == 0) huge[atomicAdd(nhuge, 1u)] = u;
            continue;
        }
        uint64_t t = 0;
        for (uint32_t j = j0 + __lane_id(); j < j1; j += WAVE) {
            const uint32_t e = inc[j];
            const uint32_t sz = pin_off[e + 1] - pin_off[e];
            if (sz >= 2) t += sz - 1;
        }
        t = wave_sum(t);
        if (__lane_id() == 0) bound[u] = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
    }
}

// Fill cursors of the candidate lists: the exclusive prefix of the nk
// (sub-round, class) counts (one workgroup), the same offsets the host forms
// from its read-back of the counts.
__global__ __launch_bounds__(BLOCK) void k_class_offsets(const uint32_t *counts, uint32_t nk, uint32_t *cursor) {
    __shared__ uint32_t wsum[BLOCK / WAVE];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nk; b += BLOCK) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < nk ? counts[i] : 0u;
        uint32_t tot;
        const uint32_t incl = block_incl_scan<uint32_t>(v, wsum, &tot);
        if (i < nk) cursor[i] = carry + incl - v;
        carry += tot;
    }
}

// Sets one device word from a host value (a kernel argument instead of a
// copy from pageable host memory, which would be a host round trip).
__global__ void k_put_word(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// pass 1 (fill=false): count per (sub-round, class); pass 2: fill lists.
// Counters are aggregated per block in LDS: each block adds its counts with
// one global atomic per key (and in pass 2 reserves its ranges the same way),
// so millions of vertices never contend on a handful of addresses.  At most
// CLASSIFY_BLOCKS blocks, since atomics on one address are serialised.
constexpr int MAX_KEYS = 256 * NCLASS;
constexpr unsigned CLASSIFY_BLOCKS = 512;
// The class of a candidate follows D = min(B(u), n - 1), a bound on the
// distinct clusters it rates; counts[S * NCLASS] receives the largest D of
// the global-table class and counts[S * NCLASS + 2] the largest vertex weight.
__device__ inline int classify_key(const uint32_t *bound, uint32_t n, uint64_t mseed, uint32_t level, uint32_t S,
                                   uint32_t u, uint32_t *D) {
    *D = bound[u] < n - 1 ? bound[u] : n - 1;
    const int c = rate_class(*D);
    if (c < 0) return -1;
    return (int)((uint32_t)(tag_hash(mseed, 1, level, 0, u) % S) * NCLASS + c);
}

// Block b takes the contiguous vertex range [b * per, (b + 1) * per), and its
// vertices of each key go to the list after those of blocks 0 .. b-1 (per-
// block counts of pass 1 in bcounts[key * gridDim + b]), so every list holds
// its vertices about in ascending order: the rating kernels give each XCD a
// contiguous part of a list, hence of the vertex range.
__global__ __launch_bounds__(BLOCK) void k_classify(const uint32_t *bound, uint32_t n, uint64_t mseed,
                                                    uint32_t level, uint32_t S, const int32_t *vwgt, uint32_t *rep,
                                                    int64_t *cw, int64_t *tsum, uint32_t *counts, uint32_t *cursor,
                                                    uint32_t *bcounts, uint32_t *lists, bool fill) {
    __shared__ uint32_t lcnt[MAX_KEYS];
    __shared__ uint32_t lbase[MAX_KEYS];
    __shared__ uint32_t lmaxd, lmaxw;
    const uint32_t nkeys = S * NCLASS;
    for (uint32_t i = threadIdx.x; i < nkeys; i += BLOCK) lcnt[i] = 0;
    if (threadIdx.x == 0) { lmaxd = 0; lmaxw = 0; }
    __syncthreads();
    uint32_t mw = 0;  // largest vertex weight seen by the thread
    const uint32_t per = (uint32_t)(((uint64_t)n + gridDim.x - 1) / gridDim.x);
    const uint32_t ulo = (uint32_t)min((uint64_t)blockIdx.x * per, (uint64_t)n);
    const uint32_t uhi = (uint32_t)min((uint64_t)ulo + per, (uint64_t)n);
    for (uint32_t u = ulo + threadIdx.x; u < uhi; u += BLOCK) {
        uint32_t D;
        const int key = classify_key(bound, n, mseed, level, S, u, &D);
        if (!fill) {
            const int32_t w = vwgt[u];
            rep[u] = u;
            cw[u] = w;
            tsum[u] = 0;
            mw = (uint32_t)w > mw ? (uint32_t)w : mw;
            if (key >= 0 && (uint32_t)key % NCLASS == NCLASS - 1) atomicMax(&lmaxd, D);
        }
        if (key >= 0) atomicAdd(&lcnt[key], 1u);
    }
    if (!fill) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t y = __shfl_xor(mw, o, 64);
            mw = y > mw ? y : mw;
        }
        if (__lane_id() == 0 && mw) atomicMax(&lmaxw, mw);
    }
    __syncthreads();
    if (!fill) {
        for (uint32_t i = threadIdx.x; i < nkeys; i += BLOCK) {
            if (lcnt[i]) atomicAdd(&counts[i], lcnt[i]);
            bcounts[(size_t)i * gridDim.x + blockIdx.x] = lcnt[i];
        }
        if (threadIdx.x == 0 && lmaxd) atomicMax(&counts[nkeys], lmaxd);
        if (threadIdx.x == 0 && lmaxw) atomicMax(&counts[nkeys + 2], lmaxw);
        return;
    }
    for (uint32_t i = threadIdx.x; i < nkeys; i += BLOCK) {
        uint32_t before = cursor[i];  // the list's start
        for (uint32_t b = 0; b < blockIdx.x; ++b) before += bcounts[(size_t)i * gridDim.x + b];
        lbase[i] = before;
        lcnt[i] = 0;
    }
    __syncthreads();
    for (uint32_t u = ulo + threadIdx.x; u < uhi; u += BLOCK) {
        uint32_t D;
        const int key = classify_key(bound, n, mseed, level, S, u, &D);
        if (key >= 0) lists[lbase[key] + atomicAdd(&lcnt[key], 1u)] = u;
    }
}

// ---------------------------------------------------------------------------
// Approval and apply
// ---------------------------------------------------------------------------
// Proposers are the candidates of the sub-round's list whose target is set.
__global__ void k_approve_fast(const uint32_t *cands, uint32_t nc, const uint32_t *ptarget, const int64_t *cw,
                               const int64_t *tsum, int64_t cap_mult, int64_t W, uint8_t *ok, uint32_t *slow,
                               uint32_t *nslow, const uint32_t *ncl, uint32_t n, const uint32_t *ovf) {
    if (ovf_set(ovf) || pass_cut(ncl, n)) return;  // nothing was rated
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ((nc + 63) / 64) * 64;
         i += gridDim.x * blockDim.x) {
        const uint32_t u = i < nc ? cands[i] : 0;
        const uint32_t C = i < nc ? ptarget[u] : NONE;
        const bool act = C != NONE;
        bool fits = true;
        if (act) {
            fits = cap_mult * (cw[C] + tsum[C]) <= W;
            ok[u] = fits ? 1 : 0;
        }
        uint32_t pos = warp_agg_append(nslow, act && !fits);
        if (act && !fits) slow[pos] = u;
    }
}

// key = (C << (wb + ub)) | (c(u) << ub) | u  when it fits in 64 bits
__global__ void k_slow_keys(const uint32_t *slow, uint32_t ns, const uint32_t *ptarget, const int32_t *vwgt,
                            int wb, int ub, uint64_t *keys, uint32_t *vals, bool with_u) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        uint32_t u = slow[i];
        uint64_t key = ((uint64_t)ptarget[u] << (wb + (with_u ? ub : 0))) |
                       ((uint64_t)(uint32_t)vwgt[u] << (with_u ? ub : 0)) | (with_u ? (uint64_t)u : 0);
        keys[i] = key;
        vals[i] = u;
    }
}

__global__ void k_u_keys(const uint32_t *slow, uint32_t ns, uint64_t *keys, uint32_t *vals) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        keys[i] = slow[i];
        vals[i] = slow[i];
    }
}

// Sorted slow joins: segment start of each target writes the base prefix.
struct WeightOfSorted {
    const uint32_t *vals;
    const int32_t *vwgt;
    __device__ uint64_t operator()(size_t i) const { return (uint64_t)(uint32_t)vwgt[vals[i]]; }
};
struct StoreInclU64 {
    uint64_t *out;
    __device__ void operator()(size_t i, uint64_t excl, uint64_t v) const { out[i] = excl + v; }
};

__global__ void k_slow_decide(const uint32_t *vals, uint32_t ns, const uint32_t *ptarget, const uint64_t *incl,
                              const int32_t *vwgt, const int64_t *cw, int64_t cap_mult, int64_t W, uint8_t *ok) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        uint32_t u = vals[i];
        uint32_t C = ptarget[u];
        // find the segment start by walking back over equal targets is O(len);
        // instead binary search: segments are contiguous, sorted by C.
        uint32_t lo = 0, hi = i;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (ptarget[vals[mid]] < C) lo = mid + 1; else hi = mid;
        }
        uint64_t base = lo == 0 ? 0 : incl[lo - 1];
        int64_t prefix = (int64_t)(incl[i] - base);
        ok[u] = (cap_mult * (cw[C] + prefix) <= W) ? 1 : 0;
    }
}

// The sorted approval of up to SLOW_SMALL joins in one workgroup: keys
// (C, c(u), u) sorted in LDS (bitonic), prefix sums of c(u), and the same
// decision as k_slow_decide.  Needs the key to fit 64 bits.
constexpr uint32_t SLOW_SMALL = 4096;
constexpr int SLOW_THREADS = 1024;
// With ns_dev the count is read on the device (queued passes): nothing to do
// when the sub-round found the pass cut or an earlier one awaits the host,
// and more than SLOW_SMALL joins hand the sub-round to the host (ovf).
__global__ __launch_bounds__(SLOW_THREADS) void k_slow_small(const uint32_t *slow, uint32_t ns,
                                                             const uint32_t *ptarget, const int32_t *vwgt,
                                                             const int64_t *cw, int64_t cap_mult, int64_t W,
                                                             uint8_t *ok, int wb, int ub, const uint32_t *ns_dev,
                                                             const uint32_t *cut_r, uint32_t *ovf, uint32_t r) {
    __shared__ uint64_t key[SLOW_SMALL];
    __shared__ uint64_t incl[SLOW_SMALL];
    __shared__ uint64_t wsum[SLOW_THREADS / WAVE];
    if (ns_dev) {
        if (*cut_r || *ovf) return;
        ns = *ns_dev;
        if (ns > SLOW_SMALL) {
            if (threadIdx.x == 0) *ovf = r + 1;
            return;
        }
    }
    if (ns == 0) return;
    const uint32_t tid = threadIdx.x;
    const int cs = wb + ub;
    const uint64_t umask = (1ull << ub) - 1ull, wmask = (1ull << wb) - 1ull;
    uint32_t n2 = 1;
    while (n2 < ns) n2 <<= 1;
    for (uint32_t i = tid; i < n2; i += SLOW_THREADS) {
        uint64_t k = ~0ull;
        if (i < ns) {
            const uint32_t u = slow[i];
            k = ((uint64_t)ptarget[u] << cs) | ((uint64_t)(uint32_t)vwgt[u] << ub) | (uint64_t)u;
        }
        key[i] = k;
    }
    __syncthreads();
    for (uint32_t kk = 2; kk <= n2; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < n2; i += SLOW_THREADS) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t a = key[i], b = key[l];
                    if ((a > b) == ((i & kk) == 0)) { key[i] = b; key[l] = a; }
                }
            }
            __syncthreads();
        }
    }
    uint64_t carry = 0;
    for (uint32_t c0 = 0; c0 < ns; c0 += SLOW_THREADS) {
        const uint32_t i = c0 + tid;
        const uint64_t w = i < ns ? (key[i] >> ub) & wmask : 0ull;
        uint64_t tot;
        const uint64_t inc = block_incl_scan_n<uint64_t, SLOW_THREADS>(w, wsum, &tot);
        if (i < ns) incl[i] = carry + inc;
        carry += tot;
    }
    __syncthreads();
    for (uint32_t i = tid; i < ns; i += SLOW_THREADS) {
        const uint64_t C = key[i] >> cs;
        uint32_t lo = 0, hi = i;  // first position of target C
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((key[mid] >> cs) < C) lo = mid + 1; else hi = mid;
        }
        const uint64_t base = lo == 0 ? 0 : incl[lo - 1];
        const int64_t prefix = (int64_t)(incl[i] - base);
        ok[(uint32_t)(key[i] & umask)] = (cap_mult * (cw[C] + prefix) <= W) ? 1 : 0;
    }
}

// The joins of a block are counted in LDS and leave the cluster count with
// one atomic per block (APPLY_BLOCKS at most).
constexpr unsigned APPLY_BLOCKS = 512;
__global__ __launch_bounds__(BLOCK) void k_apply_joins(const uint32_t *cands, uint32_t nc, const uint32_t *ptarget,
                                                       const uint8_t *ok, const int32_t *vwgt, uint32_t *rep,
                                                       int64_t *cw, int64_t *tsum, uint32_t *n_clusters,
                                                       const uint32_t *cut_r, const uint32_t *ovf) {
    __shared__ uint32_t red[BLOCK / WAVE];
    if (*cut_r || ovf_set(ovf)) return;  // nothing was rated, or the host finishes the sub-round
    uint32_t joins = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        const uint32_t u = cands[i];
        const uint32_t C = ptarget[u];
        if (C == NONE) continue;
        tsum[C] = 0;
        if (ok[u]) {
            ++joins;
            rep[u] = C;
            atomic_add_i64(&cw[C], (int64_t)vwgt[u]);
        }
    }
    joins = wave_sum(joins);
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = joins;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
        if (t) atomicSub(n_clusters, t);
    }
}

// ---------------------------------------------------------------------------
// Host driver of one pass
// ---------------------------------------------------------------------------
struct CoarsenBufs {
    uint64_t *nscore;
    int64_t *cw, *tsum, *tinfo;
    uint32_t *ptarget, *slow, *lists, *counts, *cursor, *bcounts, *scal;
    uint8_t *ok;
    uint64_t *keys, *keys_alt, *incl;
    uint32_t *vals, *vals_alt;
    uint32_t *bound;
    char *greg;         // region of the global (hub) rating tables
    size_t greg_bytes;  // at least 16 tables for the worst case D = n - 1
    uint4 *hub_info;
    HubJob *hub_jobs;
    HubItem *hub_items;
    size_t hub_items_cap;
    HubItem *hub_aitems;     // argmax slices of one batch
    size_t hub_aitems_cap;
    uint64_t *hub_partR;     // best target per slice
    uint32_t *hub_partC;
    uint32_t *hub_ovf;       // [n + 1]: LDS jobs whose table filled up (flags), their count last
    uint32_t *hub_ovf_list;  // [n]
};

// One global-table entry: key, stamp (4 B each), rating (8 B).
constexpr size_t GENTRY_BYTES = 16;

static void plan(Arena &A, uint32_t n, uint32_t m, uint32_t p, uint32_t S, CoarsenBufs &B) {
    B.nscore = A.alloc<uint64_t>(m);
    B.cw = A.alloc<int64_t>(n);
    B.tsum = A.alloc<int64_t>(n);
    B.tinfo = A.alloc<int64_t>(n);
    B.ptarget = A.alloc<uint32_t>(n);
    B.slow = A.alloc<uint32_t>(n);
    B.lists = A.alloc<uint32_t>(n);
    // + largest D, largest net, largest vertex weight, vertices of more than VB_HUGE nets
    B.counts = A.alloc<uint32_t>((size_t)S * NCLASS + 4);
    B.bound = A.alloc<uint32_t>(n);
    B.cursor = A.alloc<uint32_t>((size_t)S * NCLASS);
    B.bcounts = A.alloc<uint32_t>((size_t)S * NCLASS * CLASSIFY_BLOCKS);
    B.scal = A.alloc<uint32_t>(8 + 256);  // counters, then the cut decision of every sub-round
    B.ok = A.alloc<uint8_t>(n);
    B.keys = A.alloc<uint64_t>(n);
    B.keys_alt = A.alloc<uint64_t>(n);
    B.incl = A.alloc<uint64_t>(n);
    B.vals = A.alloc<uint32_t>(n);
    B.vals_alt = A.alloc<uint32_t>(n);
    B.hub_info = A.alloc<uint4>(n);
    B.hub_jobs = A.alloc<HubJob>(n);
    B.hub_items_cap = (size_t)p / HUB_MIN_NETS + n + 1;
    B.hub_items = A.alloc<HubItem>(B.hub_items_cap);
    // argmax slices of one batch: a batch's tables fit the region (at most
    // 2^26 entries), so it has at most one slice per job plus one per
    // ARG_SLICE entries of the region
    B.hub_aitems_cap = (size_t)n + ((size_t)1 << 26) / ARG_SLICE + 1;
    B.hub_aitems = A.alloc<HubItem>(B.hub_aitems_cap);
    B.hub_partR = A.alloc<uint64_t>(B.hub_aitems_cap);
    B.hub_partC = A.alloc<uint32_t>(B.hub_aitems_cap);
    B.hub_ovf = A.alloc<uint32_t>((size_t)n + 1);
    B.hub_ovf_list = A.alloc<uint32_t>(n);
    // global (hub) rating tables: room for 16 tables of the largest possible
    // capacity (>= 1.5 n), more (up to 4 p entries, 2^26) when the workspace
    // has it, always leaving room for the temporaries the pass allocates
    // later (sorts, scans, reductions).  The region only decides how many hub
    // jobs run per batch, so a deep hierarchy that leaves less room gets a
    // smaller region, down to one largest table.
    Arena T(nullptr, 0);
    sort_reserve(T, n);
    scan_reserve<uint64_t>(T, n);
    const size_t tail = T.peak + 65536;
    size_t sc = 8192;
    while (sc < (size_t)n + n / 2 + 1) sc <<= 1;
    size_t entries = 16 * sc;
    while (entries < 4 * (size_t)p && entries < ((size_t)1 << 26)) entries <<= 1;
    const size_t rem = A.remaining();
    const size_t avail = (rem > tail ? rem - tail : 0) / GENTRY_BYTES;
    while (entries > sc && entries > avail) entries >>= 1;
    B.greg_bytes = entries * GENTRY_BYTES;
    B.greg = A.alloc<char>(B.greg_bytes);
    // radix sort temporaries (reserved and released: counted in the peak)
    sort_reserve(A, n);
    scan_reserve<uint64_t>(A, n);
}

size_t coarsen_workspace(uint32_t n, uint32_t m, uint32_t p, const hgp_params &prm) {
    Arena A(nullptr, 0);
    CoarsenBufs B;
    plan(A, n, m, p, prm.coarsen_subrounds, B);
    return A.peak;
}

void coarsen_pass(const hgp_hg &h, const hgp_params &prm, uint32_t level, uint32_t *rep, uint32_t *n_clusters_dev,
                  uint32_t *n_clusters_host, Arena &A, hipStream_t st, int64_t W_known, const uint32_t *comm) {
    const uint32_t n = h.n, m = h.m, S = prm.coarsen_subrounds;
    size_t mk = A.mark();
    CoarsenBufs B;
    plan(A, n, m, h.p, S, B);
    // c(V) is needed on the host for the cap test constants
    const int64_t W = W_known >= 0 ? W_known : total_weight(h.vwgt, n, A, st);
    const int64_t cap_mult = (int64_t)prm.limit_factor * (int64_t)prm.k;
    const uint64_t mseed = mix64(prm.seed);

    k_net_score<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.nwgt, m, B.nscore);
    HGP_LAUNCH_CHECK();
    HGP_CHECK_HIP(hipMemsetAsync(B.counts, 0, sizeof(uint32_t) * (S * NCLASS + 4), st));
    uint32_t *nhuge = B.counts + S * NCLASS + 3;
    if ((uint64_t)h.p >= (uint64_t)16 * n)  // average degree of at least 16: a wave per vertex
        k_vertex_b_wave<<<grid_for((size_t)std::max(n, m) * WAVE, BLOCK, 4 * FILL_BLOCKS), BLOCK, 0, st>>>(
            h.pin_off, h.inc_off, h.inc, n, m, B.bound, B.counts + S * NCLASS + 1, B.slow, nhuge);
    else
        k_vertex_b<<<grid_for(std::max(n, m), BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
            h.pin_off, h.inc_off, h.inc, n, m, B.bound, B.counts + S * NCLASS + 1, B.slow, nhuge);
    HGP_LAUNCH_CHECK();
    if ((uint64_t)h.p > VB_HUGE) {  // a vertex of more than VB_HUGE nets can exist
        k_vertex_b_huge<<<256, VB_HUGE_THREADS, 0, st>>>(h.pin_off, h.inc_off, h.inc, B.slow, nhuge, B.bound);
        HGP_LAUNCH_CHECK();
    }
    k_classify<<<grid_for(n, BLOCK, CLASSIFY_BLOCKS), BLOCK, 0, st>>>(B.bound, n, mseed, level, S, h.vwgt, rep, B.cw,
                                                                 B.tsum, B.counts, B.cursor, B.bcounts, B.lists, false);
    HGP_LAUNCH_CHECK();
    std::vector<uint32_t> counts(S * NCLASS + 3), offs(S * NCLASS + 1);
    read_back(counts.data(), B.counts, sizeof(uint32_t) * (S * NCLASS + 3), st);
    const bool huge_nets = counts[S * NCLASS + 1] > HUB_BIG;
    const bool small_nets = counts[S * NCLASS + 1] <= 8;  // every net fits the 8-pin lane path
    // hub tables: the whole region, cleared once; every job leaves its slots clean
    const size_t E = B.greg_bytes / GENTRY_BYTES;
    uint64_t *gR = (uint64_t *)B.greg;
    uint32_t *gkeys = (uint32_t *)(B.greg + 8 * E), *gstamp = gkeys + E;
    bool any_hub = false;
    for (uint32_t r = 0; r < S; ++r) any_hub |= counts[r * NCLASS + NCLASS - 1] > 0;
    if (any_hub) {
        HGP_CHECK_HIP(hipMemsetAsync(gR, 0, 8 * E, st));
        HGP_CHECK_HIP(hipMemsetAsync(gkeys, 0xFF, 8 * E, st));  // keys and stamps
    }
    // Measurement only: compulsory bytes of rating the jobs' candidates.
    auto account_jobs = [&](int kid, const RateArgs &a, const HubJob *jobs, uint32_t nj) {
        if (!accounting(kid) || nj == 0) return;
        Timing &T = timing();
        ++T.stamp;
        k_account_rate<<<grid_for(nj, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
            a, JobVertex{jobs}, nj, T.marks, T.marks + T.marks_len, T.marks + 2 * T.marks_len, T.stamp,
            (unsigned long long *)T.acc_dev + kid);
        HGP_LAUNCH_CHECK();
    };
    // Hub rating of the listed candidates: jobs packed into the region in
    // batches (every table fits the region alone: E >= 16 * its capacity).
    auto global_rate = [&](const RateArgs &a, const std::vector<uint4> &info) {
        const uint32_t cntc = (uint32_t)info.size();
        // all batches planned at once: jobs of a batch share the region
        std::vector<HubJob> jobs;
        std::vector<HubItem> items, aitems;
        std::vector<uint32_t> bj{0}, bi{0}, ba{0};  // batch boundaries in jobs / items / argmax slices
        size_t used = 0;
        uint32_t pb = 0;  // partial results of the batch so far
        for (uint32_t i = 0; i < cntc; ++i) {
            const uint4 f = info[i];
            if (f.w == NONE) continue;  // joined by another vertex earlier in the pass
            uint32_t lg = 13;
            while (((uint64_t)1 << lg) < (uint64_t)f.w + f.w / 2 + 1) ++lg;
            const size_t cap = (size_t)1 << lg;
            if (used + cap > E) {
                bj.push_back((uint32_t)jobs.size());
                bi.push_back((uint32_t)items.size());
                ba.push_back((uint32_t)aitems.size());
                used = 0;
                pb = 0;
            }
            const uint32_t jid = (uint32_t)(jobs.size() - bj.back());  // index within the batch
            // the argmax reads the whole table (slots left empty are skipped)
            const uint32_t nsl = (uint32_t)((cap + ARG_SLICE - 1) / ARG_SLICE);
            jobs.push_back(HubJob{f.x, lg, f.y, f.z, used, pb, nsl});
            for (uint32_t q = 0; q < nsl; ++q) aitems.push_back(HubItem{jid, q, 0, 0});
            pb += nsl;
            // insert items of about HUB_WORK pins (by the average net size)
            const uint32_t deg = f.z - f.y;
            const uint64_t avg = deg ? std::max<uint64_t>(1, (uint64_t)f.w / deg) : 1;
            const uint32_t per = (uint32_t)std::min<uint64_t>(
                HUB_CHUNK, std::max<uint64_t>(HUB_MIN_NETS, HUB_WORK / avg));
            for (uint32_t j = f.y; j < f.z; j += per)
                items.push_back(HubItem{jid, j, std::min(j + per, f.z), 0});
            used += cap;
        }
        bj.push_back((uint32_t)jobs.size());
        bi.push_back((uint32_t)items.size());
        ba.push_back((uint32_t)aitems.size());
        if (jobs.empty()) return;
        if (items.size() > B.hub_items_cap || jobs.size() > n) throw Error{HGP_E_WORKSPACE};
        HGP_CHECK_HIP(hipMemcpyAsync(B.hub_jobs, jobs.data(), sizeof(HubJob) * jobs.size(), hipMemcpyHostToDevice,
                                     st));
        HGP_CHECK_HIP(hipMemcpyAsync(B.hub_items, items.data(), sizeof(HubItem) * items.size(),
                                     hipMemcpyHostToDevice, st));
        account_jobs(KID_HUB_INSERT, a, B.hub_jobs, (uint32_t)jobs.size());
        for (size_t b = 0; b + 1 < bj.size(); ++b) {
            const uint32_t nj = bj[b + 1] - bj[b], ni = bi[b + 1] - bi[b], na = ba[b + 1] - ba[b];
            if (!nj) continue;
            if (na > B.hub_aitems_cap) throw Error{HGP_E_WORKSPACE};
            const HubJob *jb = B.hub_jobs + bj[b];
            HGP_CHECK_HIP(hipMemcpyAsync(B.hub_aitems, aitems.data() + ba[b], sizeof(HubItem) * na,
                                         hipMemcpyHostToDevice, st));
            {
                TimedLaunch tl(KID_HUB_INSERT, st);
                k_hub_insert<<<std::min(ni, 8192u), BLOCK, 0, st>>>(a, jb, B.hub_items + bi[b], ni, gkeys, gR);
                HGP_LAUNCH_CHECK();
            }
            if (huge_nets) {
                k_hub_huge<<<std::min(nj, 8192u), BLOCK, 0, st>>>(a, jb, nj, gkeys, gstamp, gR);
                HGP_LAUNCH_CHECK();
            }
            {
                TimedLaunch tl(KID_HUB_ARGMAX, st);
                k_hub_argmax<<<std::min(na, 8192u), BLOCK, 0, st>>>(a, jb, B.hub_aitems, na, gkeys, gstamp, gR,
                                                                    B.hub_partR, B.hub_partC);
                HGP_LAUNCH_CHECK();
            }
            k_hub_pick<<<grid_for((size_t)nj * WAVE, BLOCK, 1024), BLOCK, 0, st>>>(a, jb, nj, B.hub_partR,
                                                                                  B.hub_partC, nullptr);
            HGP_LAUNCH_CHECK();
        }
        stream_sync(st);  // the uploads read the host vectors
    };
    // Hub candidates: bounds up to LHUB_PART * LHUB_MAXP take the LDS path
    // (unless the level has nets of more than HUB_BIG pins), the others and
    // any LDS job whose table filled up the global-table path.
    auto hub_rate = [&](const RateArgs &a, const uint32_t *lst, uint32_t cntc) {
        k_hub_info<<<grid_for(cntc, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(a, lst, cntc, B.bound, n, B.hub_info);
        HGP_LAUNCH_CHECK();
        std::vector<uint4> info(cntc), ginfo, linfo;
        read_back(info.data(), B.hub_info, sizeof(uint4) * cntc, st);
        for (const uint4 &f : info) {
            if (f.w == NONE) continue;  // joined by another vertex earlier in the pass
            if (!huge_nets && f.w <= LHUB_PART * LHUB_MAXP) linfo.push_back(f);
            else ginfo.push_back(f);
        }
        std::vector<HubJob> ljobs;
        std::vector<HubItem> litems;
        std::vector<uint32_t> lj{0}, la{0};  // batch boundaries in jobs / items (partials <= hub_aitems_cap)
        if (!linfo.empty()) {
            uint32_t pb = 0;
            for (const uint4 &f : linfo) {
                const uint32_t P = std::max<uint32_t>(1u, (f.w + LHUB_PART - 1) / LHUB_PART);
                if (pb + P > B.hub_aitems_cap) {
                    lj.push_back((uint32_t)ljobs.size());
                    la.push_back((uint32_t)litems.size());
                    pb = 0;
                }
                const uint32_t jid = (uint32_t)(ljobs.size() - lj.back());
                ljobs.push_back(HubJob{f.x, P, f.y, f.z, 0, pb, P});
                for (uint32_t q = 0; q < P; ++q) litems.push_back(HubItem{jid, q, 0, 0});
                pb += P;
            }
            lj.push_back((uint32_t)ljobs.size());
            la.push_back((uint32_t)litems.size());
            HGP_CHECK_HIP(hipMemcpyAsync(B.hub_jobs, ljobs.data(), sizeof(HubJob) * ljobs.size(),
                                         hipMemcpyHostToDevice, st));
            account_jobs(KID_HUB_LDS, a, B.hub_jobs, (uint32_t)ljobs.size());
            HGP_CHECK_HIP(hipMemsetAsync(B.hub_ovf, 0, sizeof(uint32_t) * (ljobs.size() + 1), st));
            uint32_t *ovf_cnt = B.hub_ovf + n;
            HGP_CHECK_HIP(hipMemsetAsync(ovf_cnt, 0, sizeof(uint32_t), st));
            for (size_t b = 0; b + 1 < lj.size(); ++b) {
                const uint32_t nj = lj[b + 1] - lj[b], nl = la[b + 1] - la[b];
                if (!nj) continue;
                const HubJob *jb = B.hub_jobs + lj[b];
                HGP_CHECK_HIP(hipMemcpyAsync(B.hub_aitems, litems.data() + la[b], sizeof(HubItem) * nl,
                                             hipMemcpyHostToDevice, st));
                {
                    TimedLaunch tl(KID_HUB_LDS, st);
                    k_hub_lds<<<std::min(nl, 8192u), LHUB_THREADS, 0, st>>>(a, jb, B.hub_aitems, nl, B.hub_partR,
                                                                            B.hub_partC, B.hub_ovf + lj[b],
                                                                            B.hub_ovf_list, ovf_cnt);
                    HGP_LAUNCH_CHECK();
                }
                k_hub_pick<<<grid_for((size_t)nj * WAVE, BLOCK, 1024), BLOCK, 0, st>>>(a, jb, nj, B.hub_partR,
                                                                                      B.hub_partC, B.hub_ovf + lj[b]);
                HGP_LAUNCH_CHECK();
            }
        }
        if (!ginfo.empty()) global_rate(a, ginfo);
        if (!linfo.empty()) {
            // jobs whose LDS table filled up (indices within their batch)
            uint32_t no = 0;
            read_back(&no, B.hub_ovf + n, sizeof(uint32_t), st);
            if (no) {
                std::vector<uint32_t> flags(ljobs.size());
                HGP_CHECK_HIP(hipMemcpyAsync(flags.data(), B.hub_ovf, sizeof(uint32_t) * flags.size(),
                                             hipMemcpyDeviceToHost, st));
                stream_sync(st);
                std::vector<uint4> again;
                for (size_t q = 0; q < flags.size(); ++q)
                    if (flags[q]) again.push_back(linfo[q]);
                global_rate(a, again);
            }
        }
    };
    offs[0] = 0;
    for (uint32_t i = 0; i < S * NCLASS; ++i) offs[i + 1] = offs[i] + counts[i];
    k_class_offsets<<<1, BLOCK, 0, st>>>(B.counts, S * NCLASS, B.cursor);
    HGP_LAUNCH_CHECK();
    k_classify<<<grid_for(n, BLOCK, CLASSIFY_BLOCKS), BLOCK, 0, st>>>(B.bound, n, mseed, level, S, h.vwgt, rep, B.cw,
                                                                 B.tsum, B.counts, B.cursor, B.bcounts, B.lists, true);
    HGP_LAUNCH_CHECK();

    uint32_t cnt = n;
    uint32_t *nslow = B.scal + 1, *ncl = B.scal + 2, *ovf = B.scal + 3, *cut = B.scal + 8;  // cut: [S] words
    const int ub = bits_for(n ? n - 1 : 0), cb = ub;
    const int wb = bits_for((uint64_t)counts[S * NCLASS + 2]);  // bits of the largest vertex weight
    // Queued pass: every sub-round goes to the device at once when the
    // approval keys fit one word and no hub candidate needs host planning;
    // otherwise the host reads the slow-join count back after every sub-round.
    const bool queued = cb + wb + ub <= 64 && !any_hub;
    k_put_word<<<1, 64, 0, st>>>(ncl, cnt);
    HGP_LAUNCH_CHECK();
    if (queued) HGP_CHECK_HIP(hipMemsetAsync(ovf, 0, sizeof(uint32_t), st));
    auto rate_subround = [&](uint32_t r) {
        k_target_info<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(rep, B.cw, h.vwgt, n, mseed, level, S, r,
                                                                        B.tinfo, B.ptarget, ncl, nslow, cut,
                                                                        queued ? ovf : nullptr);
        HGP_LAUNCH_CHECK();
        RateArgs a{h.pin_off, h.pins, h.inc_off, h.inc, h.vwgt, B.nscore, rep, B.cw, B.tinfo, B.ptarget, B.tsum,
                   mseed, level, r, S, cap_mult, W, r > 0, ncl, n, queued ? ovf : nullptr, comm};
        for (int c = 0; c < NCLASS; ++c) {
            uint32_t cntc = counts[r * NCLASS + c];
            if (!cntc) continue;
            const uint32_t *lst = B.lists + offs[r * NCLASS + c];
            if (c == NCLASS - 1) {  // hub candidates: several kernels with host planning, not a timed one
                hub_rate(a, lst, cntc);
                continue;
            }
            const int kid = c == 0 ? KID_RATE_G8 : c == 1 ? KID_RATE_G16 : c == 2 ? KID_RATE_G64 : KID_RATE_BLOCK;
            if (accounting(kid)) {
                Timing &T = timing();
                ++T.stamp;
                k_account_rate<<<grid_for(cntc, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
                    a, ListVertex{lst}, cntc, T.marks, T.marks + T.marks_len, T.marks + 2 * T.marks_len, T.stamp,
                    (unsigned long long *)T.acc_dev + kid);
                HGP_LAUNCH_CHECK();
            }
            TimedLaunch tl(kid, st);
            switch (c) {
                case 0: {
                    const unsigned gb = grid_for(cntc, RATE_NT8 / 8, 8192);
                    if (small_nets)
                        k_rate_group<8, 64, 6, 8, RATE_NT8><<<gb, RATE_NT8, 0, st>>>(a, lst, cntc);
                    else
                        k_rate_group<8, 64, 6, LANE_NET, RATE_NT8><<<gb, RATE_NT8, 0, st>>>(a, lst, cntc);
                    break;
                }
                case 1: {
                    const unsigned gb = grid_for(cntc, RATE_NT / 16, 8192);
                    if (small_nets)
                        k_rate_group<16, 256, 8, 8, RATE_NT><<<gb, RATE_NT, 0, st>>>(a, lst, cntc);
                    else
                        k_rate_group<16, 256, 8, LANE_NET, RATE_NT><<<gb, RATE_NT, 0, st>>>(a, lst, cntc);
                    break;
                }
                case 2: {
                    const unsigned gb = grid_for(cntc, RATE_NT / 64, 8192);
                    if (small_nets)
                        k_rate_group<64, 1024, 10, 8, RATE_NT><<<gb, RATE_NT, 0, st>>>(a, lst, cntc);
                    else
                        k_rate_group<64, 1024, 10, LANE_NET, RATE_NT><<<gb, RATE_NT, 0, st>>>(a, lst, cntc);
                    break;
                }
                default:
                    k_rate_block<<<grid_for(cntc, 1, 8192), BLOCK, 0, st>>>(a, lst, cntc);
                    break;
            }
            HGP_LAUNCH_CHECK();
        }
    };
    auto cands_of = [&](uint32_t r) { return B.lists + offs[r * NCLASS]; };  // the sub-round's candidates
    auto cand_of = [&](uint32_t r) {  // candidates listed for the sub-round: a bound on its proposals
        uint32_t c = 0;
        for (int q = 0; q < NCLASS; ++q) c += counts[r * NCLASS + q];
        return c;
    };
    auto approve = [&](uint32_t r) {
        k_approve_fast<<<grid_for(cand_of(r), BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
            cands_of(r), cand_of(r), B.ptarget, B.cw, B.tsum, cap_mult, W, B.ok, B.slow, nslow, ncl, n,
            queued ? ovf : nullptr);
        HGP_LAUNCH_CHECK();
    };
    auto apply = [&](uint32_t r, const uint32_t *ovf_or_null) {
        k_apply_joins<<<grid_for(cand_of(r), BLOCK, APPLY_BLOCKS), BLOCK, 0, st>>>(
            cands_of(r), cand_of(r), B.ptarget, B.ok, h.vwgt, rep, B.cw, B.tsum, ncl, cut + r, ovf_or_null);
        HGP_LAUNCH_CHECK();
    };
    // sorted approval of ns slow joins on the host-driven path
    auto host_slow = [&](uint32_t ns) {
        uint64_t *kk = B.keys;
        uint32_t *vv = B.vals;
        if (ns <= SLOW_SMALL && cb + wb + ub <= 64) {
            k_slow_small<<<1, SLOW_THREADS, 0, st>>>(B.slow, ns, B.ptarget, h.vwgt, B.cw, cap_mult, W, B.ok, wb, ub,
                                                     nullptr, nullptr, nullptr, 0);
            HGP_LAUNCH_CHECK();
            return;
        }
        if (cb + wb + ub <= 64) {
            k_slow_keys<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.slow, ns, B.ptarget, h.vwgt, wb, ub, kk,
                                                                           vv, true);
            HGP_LAUNCH_CHECK();
            radix_sort_pairs<uint64_t>(A, &kk, &vv, kk == B.keys ? B.keys_alt : B.keys,
                                       vv == B.vals ? B.vals_alt : B.vals, ns, 0, cb + wb + ub, st);
        } else {
            // stable two-stage: by u, then by (C, c(u))
            k_u_keys<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.slow, ns, kk, vv);
            HGP_LAUNCH_CHECK();
            radix_sort_pairs<uint64_t>(A, &kk, &vv, B.keys_alt, B.vals_alt, ns, 0, ub, st);
            uint64_t *k2 = (kk == B.keys) ? B.keys_alt : B.keys;
            uint32_t *v2 = (vv == B.vals) ? B.vals_alt : B.vals;
            k_slow_keys<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(vv, ns, B.ptarget, h.vwgt, wb, 0, kk, v2,
                                                                           false);
            HGP_LAUNCH_CHECK();
            // kk holds keys aligned with v2 (= copy of vv)
            uint32_t *vcur = v2;
            radix_sort_pairs<uint64_t>(A, &kk, &vcur, k2, vv, ns, 0, cb + wb, st);
            vv = vcur;
        }
        scan_apply<uint64_t>(A, ns, WeightOfSorted{vv, h.vwgt}, StoreInclU64{B.incl}, (uint64_t *)nullptr, st);
        k_slow_decide<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(vv, ns, B.ptarget, B.incl, h.vwgt, B.cw,
                                                                         cap_mult, W, B.ok);
        HGP_LAUNCH_CHECK();
    };
    if (queued) {
        // one read-back per pass (more when a sub-round is handed back)
        uint32_t r0 = 0;
        for (;;) {
            for (uint32_t r = r0; r < S; ++r) {
                rate_subround(r);
                if (!cand_of(r)) {  // nothing listed: the sub-round only records its cut decision
                    continue;
                }
                approve(r);
                k_slow_small<<<1, SLOW_THREADS, 0, st>>>(B.slow, 0, B.ptarget, h.vwgt, B.cw, cap_mult, W, B.ok, wb,
                                                         ub, nslow, cut + r, ovf, r);
                HGP_LAUNCH_CHECK();
                apply(r, ovf);
            }
            uint32_t hv[2];  // cluster count, handed-back sub-round
            read_back(hv, ncl, sizeof(hv), st);
            cnt = hv[0];
            if (!hv[1]) break;
            // sub-round hv[1] - 1 had more slow joins than one workgroup
            // sorts: approve them on the host-driven path, apply, go on
            const uint32_t r = hv[1] - 1;
            uint32_t ns = 0;
            read_back(&ns, nslow, sizeof(uint32_t), st);
            HGP_CHECK_HIP(hipMemsetAsync(ovf, 0, sizeof(uint32_t), st));
            host_slow(ns);
            apply(r, nullptr);
            r0 = r + 1;
        }
    } else {
        for (uint32_t r = 0; r < S; ++r) {
            rate_subround(r);
            if (!cand_of(r)) continue;
            approve(r);
            // one read-back per sub-round: the joins that need the sorted
            // approval, and the cluster count after the previous sub-round
            uint32_t hv[3];
            read_back(hv, B.scal, sizeof(hv), st);
            const uint32_t ns = hv[1];
            cnt = hv[2];
            if ((uint64_t)5 * cnt < (uint64_t)2 * n) break;  // the pass was cut: nothing was proposed
            if (ns) host_slow(ns);
            apply(r, nullptr);
        }
        read_back(&cnt, ncl, sizeof(uint32_t), st);
    }
    if (n_clusters_dev)
        HGP_CHECK_HIP(hipMemcpyAsync(n_clusters_dev, ncl, sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    if (n_clusters_host) *n_clusters_host = cnt;
    A.release(mk);
}

}  // namespace hgp
