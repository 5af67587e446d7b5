// Gain table of a partition (paper Sec. 6.2) and the gains of a move
// sequence (Sec. 6.3, the parallel gain recalculation).
//
//  - benefit b(u) = w({e in I(u): Phi(e, Pi[u]) = 1}), penalty p(u, t) =
//    w({e in I(u): Phi(e, t) = 0}); the gain of moving u to t is b(u) - p(u, t).
//    Stored as int32 (every weight sum is below 2^31): benefit[n] and
//    penalty[n * k], row u holding the k penalties of u.
//  - The table is built from the connectivity sets of the nets: Lambda(e)
//    (blocks with a pin of e) and Lambda1(e) (blocks with exactly one pin),
//    k-bit sets computed once per call.  A wave takes batches of consecutive
//    vertices whose nets fill its 64 lanes (all loads of a batch at once),
//    and every lane adds the weights of a vertex's nets whose Lambda holds
//    its block, so a row of penalties leaves as one coalesced store.
//  - A batch of moves is applied net by net: the first mover to reach a net
//    claims it (a per-net stamp) and compares Phi(e, .) before and after the
//    batch; a block whose count crosses zero changes the penalty of every pin
//    of e, a block whose count crosses one changes the benefit of its
//    unmoved pins.  Integer atomics make the result independent of the order
//    (it is the table of the new partition); the movers' benefits are
//    recomputed afterwards, as in the paper.
//  - The sequence gains follow the recalculation of Sec. 6.3 per claimed net:
//    for each block, the first move into it and the last move out of it among
//    the net's pins and the number of unmoved pins in it decide which moves
//    remove the net from a block (+w) or add it to one (-w).
//  Nets of up to SMALL_NET pins are handled by the claiming lane with
//  quadratic loops over the pins; longer nets are listed and handled by a
//  wave each with per-block counters in LDS.
#include "kernels.h"
#include "prims.h"

#include <algorithm>

namespace hgp {

namespace {

constexpr uint32_t SMALL_NET = 32;

// Lambda and Lambda1 words of a net, from the blocks of its pins.
template <int KW>
__device__ inline void fold_block(uint32_t b, uint64_t *once, uint64_t *twice) {
#pragma unroll
    for (int q = 0; q < KW; ++q) {
        const uint64_t bit = ((uint32_t)q == (b >> 6)) ? (1ull << (b & 63)) : 0ull;
        twice[q] |= once[q] & bit;
        once[q] |= bit;
    }
}

// Thread per net up to SMALL_NET pins; longer nets are listed for a wave each.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_gt_conn(const uint32_t *pin_off, const uint32_t *pins, uint32_t m,
                                                   const uint32_t *part, uint64_t *lam, uint64_t *lam1,
                                                   uint32_t *longl, uint32_t *nlong) {
    for (uint32_t e = blockIdx.x * BLOCK + threadIdx.x; e < m; e += gridDim.x * BLOCK) {
        const uint32_t b = pin_off[e], len = pin_off[e + 1] - b;
        if (len > SMALL_NET) {
            longl[atomicAdd(nlong, 1u)] = e;
            continue;
        }
        uint64_t once[KW], twice[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) { once[q] = 0; twice[q] = 0; }
        for (uint32_t j = 0; j < len; ++j) fold_block<KW>(part[pins[b + j]], once, twice);
#pragma unroll
        for (int q = 0; q < KW; ++q) {
            lam[(size_t)e * KW + q] = once[q];
            lam1[(size_t)e * KW + q] = once[q] & ~twice[q];
        }
    }
}

template <int KW>
__global__ __launch_bounds__(BLOCK) void k_gt_conn_long(const uint32_t *pin_off, const uint32_t *pins,
                                                        const uint32_t *longl, const uint32_t *nlong,
                                                        const uint32_t *part, uint64_t *lam, uint64_t *lam1) {
    const uint32_t nl = *nlong, lane = __lane_id();
    const uint32_t w0 = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE, nw = gridDim.x * (BLOCK / WAVE);
    for (uint32_t i = w0; i < nl; i += nw) {
        const uint32_t e = longl[i], b = pin_off[e], len = pin_off[e + 1] - b;
        uint64_t once[KW], twice[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) { once[q] = 0; twice[q] = 0; }
        for (uint32_t j = lane; j < len; j += WAVE) fold_block<KW>(part[pins[b + j]], once, twice);
        // (once, twice) pairs combine as once = o1 | o2, twice = t1 | t2 | (o1 & o2)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint64_t oo = __shfl_xor(once[q], o, WAVE), ot = __shfl_xor(twice[q], o, WAVE);
                twice[q] |= ot | (once[q] & oo);
                once[q] |= oo;
            }
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                lam[(size_t)e * KW + q] = once[q];
                lam1[(size_t)e * KW + q] = once[q] & ~twice[q];
            }
    }
}

// Wave-uniform reads of lane c's registers (c uniform): no LDS traffic.
__device__ inline int32_t lane_i32(int32_t v, uint32_t c) { return __builtin_amdgcn_readlane(v, (int)c); }
__device__ inline uint64_t lane_u64(uint64_t v, uint32_t c) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)c);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)c);
    return ((uint64_t)hi << 32) | lo;
}

// A wave per contiguous range of vertices.  Each step takes the next batch
// of consecutive vertices whose incident nets fit the 64 lanes (one net per
// lane: its weight, its Lambda words and the Lambda1 bit of its vertex's
// block, all loaded at once), then writes the batch's rows one vertex after
// the other: lane l owns blocks q * 64 + l and adds the weights of the
// vertex's nets whose Lambda holds its block (wave-uniform register reads),
// so every row leaves as one coalesced store.  A vertex of more than 64 nets
// is a batch of its own, walked 64 nets at a time.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_gt_rows(const uint32_t *inc_off, const uint32_t *inc, const int32_t *nwgt,
                                                   const uint32_t *part, const uint64_t *lam, const uint64_t *lam1,
                                                   uint32_t n, uint32_t k, int32_t *ben, int32_t *pen) {
    const uint32_t lane = __lane_id();
    const uint32_t wid = (blockIdx.x * BLOCK + threadIdx.x) / WAVE, nwv = gridDim.x * (BLOCK / WAVE);
    const uint32_t per = (uint32_t)(((uint64_t)n + nwv - 1) / nwv);
    uint32_t u = (uint32_t)min((uint64_t)wid * per, (uint64_t)n);
    const uint32_t uend = (uint32_t)min((uint64_t)u + per, (uint64_t)n);
    while (u < uend) {  // uniform per wave
        // degrees of the next 64 vertices and their inclusive prefix
        const uint32_t cand = u + lane;
        uint32_t o = 0, d = 0, blk = 0;
        if (cand < uend) {
            o = inc_off[cand];
            d = inc_off[cand + 1] - o;
            blk = part[cand];
        }
        uint32_t pre = d;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const uint32_t t = __shfl_up(pre, off, WAVE);
            if (lane >= (uint32_t)off) pre += t;
        }
        const uint64_t fit = __ballot(cand < uend && pre <= WAVE);  // a prefix of the lanes
        const uint32_t nb = (uint32_t)__popcll(fit);
        if (nb == 0) {
            // one vertex of more than 64 nets
            const uint32_t j0 = lane_i32((int32_t)o, 0), j1 = j0 + lane_i32((int32_t)d, 0);
            const uint32_t s = (uint32_t)lane_i32((int32_t)blk, 0);
            int64_t acc[KW];
#pragma unroll
            for (int q = 0; q < KW; ++q) acc[q] = 0;
            int64_t bsum = 0, wsum = 0;
            for (uint32_t c0 = j0; c0 < j1; c0 += WAVE) {
                const uint32_t j = c0 + lane;
                int32_t w = 0, bw = 0;
                uint64_t x[KW];
#pragma unroll
                for (int q = 0; q < KW; ++q) x[q] = 0;
                if (j < j1) {
                    const uint32_t e = inc[j];
                    w = nwgt[e];
#pragma unroll
                    for (int q = 0; q < KW; ++q) x[q] = lam[(size_t)e * KW + q];
                    if ((s >> 6) < (uint32_t)KW && ((lam1[(size_t)e * KW + (s >> 6)] >> (s & 63)) & 1ull)) bw = w;
                }
                const uint32_t cn = j1 - c0 < WAVE ? j1 - c0 : WAVE;
                for (uint32_t c = 0; c < cn; ++c) {
                    const int32_t wc = lane_i32(w, c);
                    wsum += wc;
                    bsum += lane_i32(bw, c);
#pragma unroll
                    for (int q = 0; q < KW; ++q)
                        if ((lane_u64(x[q], c) >> lane) & 1ull) acc[q] += wc;
                }
            }
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint32_t t = (uint32_t)q * 64 + lane;
                if (t < k) pen[(size_t)u * k + t] = (int32_t)(wsum - acc[q]);
            }
            if (lane == 0) ben[u] = (int32_t)bsum;
            u += 1;
            continue;
        }
        // slot lane j of the batch: net (j - excl) of vertex `own`, where own
        // is the first batch vertex whose inclusive prefix exceeds j
        const uint32_t total = (uint32_t)lane_i32((int32_t)pre, nb - 1);
        int32_t w = 0, bw = 0;
        uint64_t x[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) x[q] = 0;
        {
            uint32_t lo = 0, hi = nb - 1;  // first i in [0, nb) with pre_i > lane
#pragma unroll
            for (int it = 0; it < 6; ++it) {
                const uint32_t mid = (lo + hi) >> 1;
                const uint32_t pm = (uint32_t)__shfl((int)pre, (int)mid, WAVE);
                if (lo < hi) {
                    if (pm > lane) hi = mid; else lo = mid + 1;
                }
            }
            const uint32_t own = lo;
            const uint32_t po = (uint32_t)__shfl((int)pre, (int)own, WAVE);
            const uint32_t dd = (uint32_t)__shfl((int)d, (int)own, WAVE);
            const uint32_t oo = (uint32_t)__shfl((int)o, (int)own, WAVE);
            const uint32_t s = (uint32_t)__shfl((int)blk, (int)own, WAVE);
            if (lane < total) {
                const uint32_t e = inc[oo + (lane - (po - dd))];
                w = nwgt[e];
#pragma unroll
                for (int q = 0; q < KW; ++q) x[q] = lam[(size_t)e * KW + q];
                if ((s >> 6) < (uint32_t)KW && ((lam1[(size_t)e * KW + (s >> 6)] >> (s & 63)) & 1ull)) bw = w;
            }
        }
        // rows of the batch, one vertex at a time
        uint32_t c = 0;
        for (uint32_t i = 0; i < nb; ++i) {
            const uint32_t ci = c + (uint32_t)lane_i32((int32_t)d, i);
            int64_t acc[KW];
#pragma unroll
            for (int q = 0; q < KW; ++q) acc[q] = 0;
            int64_t bsum = 0, wsum = 0;
            for (; c < ci; ++c) {
                const int32_t wc = lane_i32(w, c);
                wsum += wc;
                bsum += lane_i32(bw, c);
#pragma unroll
                for (int q = 0; q < KW; ++q)
                    if ((lane_u64(x[q], c) >> lane) & 1ull) acc[q] += wc;
            }
            const uint32_t v = u + i;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint32_t t = (uint32_t)q * 64 + lane;
                if (t < k) pen[(size_t)v * k + t] = (int32_t)(wsum - acc[q]);
            }
            if (lane == 0) ben[v] = (int32_t)bsum;
        }
        u += nb;
    }
}

// Moves: idx[u] <- i for every node moved by move i (to a block other than
// its own); err[0] <- 1 on a node out of range, a target out of range or a
// node moved twice.  from[i] <- the node's block before the moves.
__global__ __launch_bounds__(BLOCK) void k_gt_mark(const uint32_t *node, const uint32_t *target, uint32_t count,
                                                   uint32_t n, uint32_t k, const uint32_t *part, uint32_t *idx,
                                                   uint32_t *from, uint32_t *err) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        const uint32_t u = node[i], t = target[i];
        if (u >= n || t >= k || part[u] >= k) { atomicOr(err, 1u); from[i] = NONE; continue; }
        const uint32_t prev = atomicCAS(&idx[u], NONE, i);
        if (prev != NONE) { atomicOr(err, 1u); from[i] = NONE; continue; }
        from[i] = part[u];
    }
}

struct MoveView {
    const uint32_t *idx;     // [n] move of the node or NONE
    const uint32_t *target;  // [count]
    const uint32_t *from;    // [count] block before the moves
    const uint32_t *part;    // [n] blocks before the moves
    // (moved, index) of v: a move to the node's own block is no move
    __device__ bool moved(uint32_t v, uint32_t *i) const {
        const uint32_t x = idx[v];
        if (x == NONE || target[x] == from[x]) return false;
        *i = x;
        return true;
    }
    __device__ uint32_t old_block(uint32_t v) const { return part[v]; }
    __device__ uint32_t new_block(uint32_t v) const {
        uint32_t i;
        return moved(v, &i) ? target[i] : part[v];
    }
};

// Claims net e for the calling lane (first mover to reach it this call).
__device__ inline bool claim(uint32_t *stamp, uint32_t e, uint32_t call) {
    return atomicCAS(&stamp[e], 0u, call) == 0u;
}

// Nets of at most TINY_NET pins: the pins' old and new blocks and move
// indices are loaded once into registers (three batches of independent
// loads), and both passes below work on the registers.
constexpr uint32_t TINY_NET = 8;
struct TinyNet {
    uint32_t v[TINY_NET], ob[TINY_NET], nb[TINY_NET], mi[TINY_NET];  // mi: move index or NONE (not moved)
};
__device__ inline void load_tiny(const MoveView &M, const uint32_t *pins, uint32_t b, uint32_t len, TinyNet &T) {
    uint32_t x[TINY_NET];
#pragma unroll
    for (uint32_t y = 0; y < TINY_NET; ++y) T.v[y] = y < len ? pins[b + y] : NONE;
#pragma unroll
    for (uint32_t y = 0; y < TINY_NET; ++y) {
        x[y] = T.v[y] != NONE ? M.idx[T.v[y]] : NONE;
        T.ob[y] = T.v[y] != NONE ? M.part[T.v[y]] : NONE;
    }
#pragma unroll
    for (uint32_t y = 0; y < TINY_NET; ++y) {
        T.nb[y] = T.ob[y];
        T.mi[y] = NONE;
        if (x[y] != NONE) {
            const uint32_t t = M.target[x[y]];
            if (t != M.from[x[y]]) { T.nb[y] = t; T.mi[y] = x[y]; }
        }
    }
}

__device__ inline void update_tiny_net(const TinyNet &T, uint32_t len, int32_t w, uint32_t k, int32_t *ben,
                                       int32_t *pen) {
#pragma unroll
    for (uint32_t x = 0; x < TINY_NET; ++x) {
        if (x >= len || T.mi[x] == NONE) continue;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint32_t blk = c == 0 ? T.ob[x] : T.nb[x];
            // judged once: at the first moved pin naming the block
            bool first = true;
            uint32_t co = 0, cn = 0;
#pragma unroll
            for (uint32_t y = 0; y < TINY_NET; ++y) {
                if (y >= len) continue;
                if (y < x && T.mi[y] != NONE && (T.ob[y] == blk || T.nb[y] == blk)) first = false;
                co += T.ob[y] == blk;
                cn += T.nb[y] == blk;
            }
            if (!first) continue;
            if ((co == 0) != (cn == 0)) {
                const int32_t d = cn == 0 ? w : -w;
#pragma unroll
                for (uint32_t y = 0; y < TINY_NET; ++y)
                    if (y < len) atomicAdd(&pen[(size_t)T.v[y] * k + blk], d);
            }
            if ((co == 1) != (cn == 1)) {
                const int32_t d = cn == 1 ? w : -w;
#pragma unroll
                for (uint32_t y = 0; y < TINY_NET; ++y)
                    if (y < len && T.mi[y] == NONE && T.ob[y] == blk) atomicAdd(&ben[T.v[y]], d);
            }
        }
    }
}

__device__ inline void recalc_tiny_net(const TinyNet &T, uint32_t len, int64_t w, unsigned long long *gain) {
#pragma unroll
    for (uint32_t x = 0; x < TINY_NET; ++x) {
        if (x >= len || T.mi[x] == NONE) continue;
        const uint32_t i = T.mi[x], s = T.ob[x], t = T.nb[x];
        int64_t last_out_s = -1, last_out_t = -1;
        uint32_t first_in_s = NONE, first_in_t = NONE, un_s = 0, un_t = 0;
#pragma unroll
        for (uint32_t y = 0; y < TINY_NET; ++y) {
            if (y >= len) continue;
            const uint32_t iy = T.mi[y];
            if (iy != NONE) {
                if (T.ob[y] == s && (int64_t)iy > last_out_s) last_out_s = iy;
                if (T.ob[y] == t && (int64_t)iy > last_out_t) last_out_t = iy;
                if (T.nb[y] == s && iy < first_in_s) first_in_s = iy;
                if (T.nb[y] == t && iy < first_in_t) first_in_t = iy;
            } else {
                un_s += T.ob[y] == s;
                un_t += T.ob[y] == t;
            }
        }
        int64_t d = 0;
        if (last_out_s == (int64_t)i && i < first_in_s && un_s == 0) d += w;
        if (first_in_t == i && (int64_t)i > last_out_t && un_t == 0) d -= w;
        if (d) atomicAdd(&gain[i], (unsigned long long)d);
    }
}

// Table update of one claimed net of at most SMALL_NET pins.
__device__ inline void update_small_net(const MoveView &M, const uint32_t *pins, uint32_t b, uint32_t len, int32_t w,
                                        uint32_t k, int32_t *ben, int32_t *pen) {
    for (uint32_t x = 0; x < len; ++x) {
        const uint32_t vx = pins[b + x];
        // the blocks that change: the old and the new block of a moved pin,
        // each judged once (at its first occurrence among the pins)
        uint32_t ix;
        if (!M.moved(vx, &ix)) continue;
        const uint32_t cand[2] = {M.from[ix], M.target[ix]};
        for (int c = 0; c < 2; ++c) {
            const uint32_t blk = cand[c];
            bool first = true;
            uint32_t co = 0, cn = 0;
            for (uint32_t y = 0; y < len; ++y) {
                const uint32_t vy = pins[b + y];
                uint32_t iy;
                const bool my = M.moved(vy, &iy);
                if (my && y < x && (M.from[iy] == blk || M.target[iy] == blk)) first = false;
                if (my && y == x && c == 1 && M.from[iy] == blk) first = false;
                co += M.old_block(vy) == blk;
                cn += (my ? M.target[iy] : M.old_block(vy)) == blk;
            }
            if (!first) continue;
            if ((co == 0) != (cn == 0)) {
                const int32_t d = cn == 0 ? w : -w;
                for (uint32_t y = 0; y < len; ++y) atomicAdd(&pen[(size_t)pins[b + y] * k + blk], d);
            }
            if ((co == 1) != (cn == 1)) {
                const int32_t d = cn == 1 ? w : -w;
                for (uint32_t y = 0; y < len; ++y) {
                    const uint32_t vy = pins[b + y];
                    uint32_t iy;
                    if (!M.moved(vy, &iy) && M.old_block(vy) == blk) atomicAdd(&ben[vy], d);
                }
            }
        }
    }
}

// Gains of the moves among the pins of one claimed net of at most SMALL_NET
// pins (the recalculation of Sec. 6.3 for this net).
__device__ inline void recalc_small_net(const MoveView &M, const uint32_t *pins, uint32_t b, uint32_t len, int64_t w,
                                        unsigned long long *gain) {
    for (uint32_t x = 0; x < len; ++x) {
        uint32_t i;
        if (!M.moved(pins[b + x], &i)) continue;
        const uint32_t s = M.from[i], t = M.target[i];
        // over the net's pins: last move out of s and of t, first move into
        // s and into t, unmoved pins in s and in t
        int64_t last_out_s = -1, last_out_t = -1;
        uint32_t first_in_s = NONE, first_in_t = NONE, un_s = 0, un_t = 0;
        for (uint32_t y = 0; y < len; ++y) {
            const uint32_t vy = pins[b + y];
            uint32_t iy;
            if (M.moved(vy, &iy)) {
                const uint32_t fy = M.from[iy], ty = M.target[iy];
                if (fy == s && (int64_t)iy > last_out_s) last_out_s = iy;
                if (fy == t && (int64_t)iy > last_out_t) last_out_t = iy;
                if (ty == s && iy < first_in_s) first_in_s = iy;
                if (ty == t && iy < first_in_t) first_in_t = iy;
            } else {
                const uint32_t by = M.old_block(vy);
                un_s += by == s;
                un_t += by == t;
            }
        }
        int64_t d = 0;
        if (last_out_s == (int64_t)i && i < first_in_s && un_s == 0) d += w;
        if (first_in_t == i && (int64_t)i > last_out_t && un_t == 0) d -= w;
        if (d) atomicAdd(&gain[i], (unsigned long long)d);
    }
}

// What a pass over the movers' nets does with each claimed net.
enum NetOp : int { OP_UPDATE = 0, OP_RECALC = 1 };

// Lane per move: the lane walks its node's nets and handles every net it
// claims (small nets at once, long nets listed).
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_gt_nets(MoveView M, const uint32_t *node, uint32_t count,
                                                   const uint32_t *inc_off, const uint32_t *inc,
                                                   const uint32_t *pin_off, const uint32_t *pins,
                                                   const int32_t *nwgt, uint32_t k, uint32_t *stamp, uint32_t call,
                                                   uint32_t *longl, uint32_t *nlong, int32_t *ben, int32_t *pen,
                                                   unsigned long long *gain) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        const uint32_t u = node[i];
        uint32_t iu;
        if (M.from[i] == NONE || !M.moved(u, &iu)) continue;
        for (uint32_t j = inc_off[u]; j < inc_off[u + 1]; ++j) {
            const uint32_t e = inc[j];
            if (!claim(stamp, e, call)) continue;
            const uint32_t b = pin_off[e], len = pin_off[e + 1] - b;
            if (len > SMALL_NET) {
                longl[atomicAdd(nlong, 1u)] = e;
                continue;
            }
            if (len <= TINY_NET) {
                TinyNet T;
                load_tiny(M, pins, b, len, T);
                if (OP == OP_UPDATE) update_tiny_net(T, len, nwgt[e], k, ben, pen);
                else recalc_tiny_net(T, len, nwgt[e], gain);
            } else if (OP == OP_UPDATE) {
                update_small_net(M, pins, b, len, nwgt[e], k, ben, pen);
            } else {
                recalc_small_net(M, pins, b, len, nwgt[e], gain);
            }
        }
    }
}

// Wave per listed long net, per-block counters in LDS.
constexpr int LW = BLOCK / WAVE;
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_gt_long(MoveView M, const uint32_t *longl, const uint32_t *nlong,
                                                   const uint32_t *pin_off, const uint32_t *pins,
                                                   const int32_t *nwgt, uint32_t k, int32_t *ben, int32_t *pen,
                                                   unsigned long long *gain) {
    // per wave: old and new pin counts (update) or first-in, last-out and
    // unmoved counts (recalculation) of every block
    __shared__ uint32_t A0[LW][256], A1[LW][256], A2[LW][256];
    const uint32_t wv = threadIdx.x / WAVE, lane = __lane_id();
    const uint32_t nl = *nlong;
    for (uint32_t li = blockIdx.x * LW + wv; li < nl; li += gridDim.x * LW) {
        const uint32_t e = longl[li], b = pin_off[e], len = pin_off[e + 1] - b;
        const int32_t w = nwgt[e];
        for (uint32_t t = lane; t < k; t += WAVE) {
            A0[wv][t] = OP == OP_UPDATE ? 0u : NONE;  // first in
            A1[wv][t] = 0u;                           // last out + 1
            A2[wv][t] = 0u;
        }
        wave_sync();
        for (uint32_t y = lane; y < len; y += WAVE) {
            const uint32_t v = pins[b + y];
            uint32_t i;
            const bool mv = M.moved(v, &i);
            const uint32_t ob = M.old_block(v);
            if (ob >= k) continue;  // blocks are < k (precondition)
            if (OP == OP_UPDATE) {
                atomicAdd(&A0[wv][ob], 1u);
                atomicAdd(&A1[wv][mv ? M.target[i] : ob], 1u);
            } else if (mv) {
                atomicMin(&A0[wv][M.target[i]], i);
                atomicMax(&A1[wv][M.from[i]], i + 1);
            } else {
                atomicAdd(&A2[wv][ob], 1u);
            }
        }
        wave_sync();
        if (OP == OP_UPDATE) {
            // penalties: blocks whose count crosses zero, for every pin
            for (uint32_t t = 0; t < k; ++t) {
                const uint32_t co = A0[wv][t], cn = A1[wv][t];
                if ((co == 0) != (cn == 0)) {
                    const int32_t d = cn == 0 ? w : -w;
                    for (uint32_t y = lane; y < len; y += WAVE) atomicAdd(&pen[(size_t)pins[b + y] * k + t], d);
                }
            }
            // benefits of unmoved pins whose block's count crosses one
            for (uint32_t y = lane; y < len; y += WAVE) {
                const uint32_t v = pins[b + y];
                uint32_t i;
                if (M.moved(v, &i)) continue;
                const uint32_t c = M.old_block(v);
                if (c >= k) continue;
                const uint32_t co = A0[wv][c], cn = A1[wv][c];
                if ((co == 1) != (cn == 1)) atomicAdd(&ben[v], cn == 1 ? w : -w);
            }
        } else {
            for (uint32_t y = lane; y < len; y += WAVE) {
                uint32_t i;
                if (!M.moved(pins[b + y], &i)) continue;
                const uint32_t s = M.from[i], t = M.target[i];
                int64_t d = 0;
                if (A1[wv][s] == i + 1 && i < A0[wv][s] && A2[wv][s] == 0) d += w;
                if (A0[wv][t] == i && (A1[wv][t] == 0 || i + 1 > A1[wv][t]) && A2[wv][t] == 0) d -= w;
                if (d) atomicAdd(&gain[i], (unsigned long long)d);
            }
        }
        wave_sync();  // the counters are cleared for the next net
    }
}

// Benefit of every mover in its new block, from the new pin counts of its nets.
__global__ __launch_bounds__(BLOCK) void k_gt_mover_benefit(MoveView M, const uint32_t *node, uint32_t count,
                                                            const uint32_t *inc_off, const uint32_t *inc,
                                                            const uint32_t *pin_off, const uint32_t *pins,
                                                            const int32_t *nwgt, int32_t *ben) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        const uint32_t u = node[i];
        uint32_t iu;
        if (M.from[i] == NONE || !M.moved(u, &iu)) continue;
        const uint32_t t = M.target[i];
        int64_t bsum = 0;
        for (uint32_t j = inc_off[u]; j < inc_off[u + 1]; ++j) {
            const uint32_t e = inc[j];
            const uint32_t b = pin_off[e], len = pin_off[e + 1] - b;
            uint32_t c = 0;
            if (len <= TINY_NET) {
                TinyNet T;
                load_tiny(M, pins, b, len, T);
#pragma unroll
                for (uint32_t y = 0; y < TINY_NET; ++y) c += y < len && T.nb[y] == t;
            } else {
                for (uint32_t q = b; q < b + len && c < 2; ++q) c += M.new_block(pins[q]) == t;
            }
            if (c == 1) bsum += nwgt[e];
        }
        ben[u] = (int32_t)bsum;
    }
}

__global__ __launch_bounds__(BLOCK) void k_gt_apply(MoveView M, const uint32_t *node, uint32_t count,
                                                    uint32_t *part) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        uint32_t iu;
        if (M.from[i] != NONE && M.moved(node[i], &iu)) part[node[i]] = M.target[i];
    }
}

// ---------------------------------------------------------------------------
// Graphs (paper Sec. 10): every net is an edge of two pins, so pin_off[e] =
// 2e and the pin array is the edge list (endpoints pins[2e], pins[2e + 1]).
// The gain table holds w(u, V_i) for every node and block (omega, int32
// [n * k]); the gain of moving u to t is omega[u][t] - omega[u][Pi[u]].
// ---------------------------------------------------------------------------

// Number of nets of other than two pins (one atomic per workgroup).
__global__ __launch_bounds__(BLOCK) void k_non_edges(const uint32_t *pin_off, uint32_t m, uint32_t *bad) {
    uint32_t c = 0;
    for (uint32_t e = blockIdx.x * BLOCK + threadIdx.x; e < m; e += gridDim.x * BLOCK)
        c += pin_off[e + 1] - pin_off[e] != 2;
    c = wave_sum(c);
    __shared__ uint32_t red[BLOCK / WAVE];
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BLOCK / WAVE; ++q) c += red[q];
        if (c) atomicAdd(bad, c);
    }
}

// Rows of omega: a wave per contiguous range of vertices, batches of
// consecutive vertices whose edges fill the 64 lanes (each lane loads one
// edge: its other endpoint's block and its weight), then every row of the
// batch is summed by the lanes that own its blocks (lane l owns blocks
// q * 64 + l) from wave-uniform register reads and leaves as one coalesced
// store.  A vertex of more than 64 edges is a batch of its own.
template <int KW>
__device__ inline void add_edge_to_row(uint32_t blk, int32_t w, uint32_t lane, int64_t (&acc)[KW]) {
#pragma unroll
    for (int q = 0; q < KW; ++q)
        if (blk == (uint32_t)q * 64 + lane) acc[q] += w;
}

template <int KW>
__global__ __launch_bounds__(BLOCK) void k_ggt_rows(const uint32_t *inc_off, const uint32_t *inc, const uint32_t *pins,
                                                    const int32_t *nwgt, const uint32_t *part, uint32_t n, uint32_t k,
                                                    int32_t *omega) {
    const uint32_t lane = __lane_id();
    const uint32_t wid = (blockIdx.x * BLOCK + threadIdx.x) / WAVE, nwv = gridDim.x * (BLOCK / WAVE);
    const uint32_t per = (uint32_t)(((uint64_t)n + nwv - 1) / nwv);
    uint32_t u = (uint32_t)min((uint64_t)wid * per, (uint64_t)n);
    const uint32_t uend = (uint32_t)min((uint64_t)u + per, (uint64_t)n);
    // the block of the other endpoint of the edge at incidence slot j of v
    auto far_block = [&](uint32_t j, uint32_t v, int32_t *w) {
        const uint32_t e = inc[j];
        const uint32_t x = pins[2 * (size_t)e], y = pins[2 * (size_t)e + 1];
        *w = nwgt[e];
        return part[x == v ? y : x];
    };
    while (u < uend) {  // uniform per wave
        const uint32_t cand = u + lane;
        uint32_t o = 0, d = 0;
        if (cand < uend) {
            o = inc_off[cand];
            d = inc_off[cand + 1] - o;
        }
        uint32_t pre = d;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const uint32_t t = __shfl_up(pre, off, WAVE);
            if (lane >= (uint32_t)off) pre += t;
        }
        const uint64_t fit = __ballot(cand < uend && pre <= WAVE);  // a prefix of the lanes
        const uint32_t nb = (uint32_t)__popcll(fit);
        if (nb == 0) {  // one vertex of more than 64 edges
            const uint32_t j0 = lane_i32((int32_t)o, 0), j1 = j0 + lane_i32((int32_t)d, 0);
            int64_t acc[KW];
#pragma unroll
            for (int q = 0; q < KW; ++q) acc[q] = 0;
            for (uint32_t c0 = j0; c0 < j1; c0 += WAVE) {
                const uint32_t j = c0 + lane;
                int32_t w = 0;
                uint32_t b = NONE;
                if (j < j1) b = far_block(j, u, &w);
                const uint32_t cn = j1 - c0 < WAVE ? j1 - c0 : WAVE;
                for (uint32_t c = 0; c < cn; ++c)
                    add_edge_to_row<KW>((uint32_t)lane_i32((int32_t)b, c), lane_i32(w, c), lane, acc);
            }
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint32_t t = (uint32_t)q * 64 + lane;
                if (t < k) omega[(size_t)u * k + t] = (int32_t)acc[q];
            }
            u += 1;
            continue;
        }
        const uint32_t total = (uint32_t)lane_i32((int32_t)pre, nb - 1);
        int32_t w = 0;
        uint32_t b = NONE;
        {
            uint32_t lo = 0, hi = nb - 1;  // first i in [0, nb) with pre_i > lane
#pragma unroll
            for (int it = 0; it < 6; ++it) {
                const uint32_t mid = (lo + hi) >> 1;
                const uint32_t pm = (uint32_t)__shfl((int)pre, (int)mid, WAVE);
                if (lo < hi) {
                    if (pm > lane) hi = mid; else lo = mid + 1;
                }
            }
            const uint32_t own = lo;
            const uint32_t po = (uint32_t)__shfl((int)pre, (int)own, WAVE);
            const uint32_t dd = (uint32_t)__shfl((int)d, (int)own, WAVE);
            const uint32_t oo = (uint32_t)__shfl((int)o, (int)own, WAVE);
            if (lane < total) b = far_block(oo + (lane - (po - dd)), u + own, &w);
        }
        uint32_t c = 0;
        for (uint32_t i = 0; i < nb; ++i) {
            const uint32_t ci = c + (uint32_t)lane_i32((int32_t)d, i);
            int64_t acc[KW];
#pragma unroll
            for (int q = 0; q < KW; ++q) acc[q] = 0;
            for (; c < ci; ++c) add_edge_to_row<KW>((uint32_t)lane_i32((int32_t)b, c), lane_i32(w, c), lane, acc);
            const uint32_t v = u + i;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint32_t t = (uint32_t)q * 64 + lane;
                if (t < k) omega[(size_t)v * k + t] = (int32_t)acc[q];
            }
        }
        u += nb;
    }
}

// Moves on a graph, in index order.  For move i (u: s -> t) and an edge
// {u, v}: v stands in target[j] when its move j comes before i, else in its
// block before the moves (M.moved and the node -> move index map decide, so
// the caller's order settles which of an edge's two moves is first).  The
// move is attributed +w when the edge stops being cut and -w when it starts
// being cut; the neighbour rows change by +w at t and -w at s (integer
// atomics: any order gives the same table).  A lane per move of up to 32
// edges, a wave per larger move.
__device__ inline void graph_edge(const MoveView &M, uint32_t i, uint32_t u, uint32_t s, uint32_t t, uint32_t e,
                                  const uint32_t *pins, const int32_t *nwgt, uint32_t k, int32_t *omega,
                                  int64_t *g) {
    const uint32_t x = pins[2 * (size_t)e], y = pins[2 * (size_t)e + 1];
    const uint32_t v = x == u ? y : x;
    const int32_t w = nwgt[e];
    uint32_t jv;
    const uint32_t bv = (M.moved(v, &jv) && jv < i) ? M.target[jv] : M.part[v];
    const bool was = bv != s, now = bv != t;
    if (was && !now) *g += w;
    if (!was && now) *g -= w;
    if (omega) {
        atomicAdd(&omega[(size_t)v * k + t], w);
        atomicAdd(&omega[(size_t)v * k + s], -w);
    }
}

__global__ __launch_bounds__(BLOCK) void k_graph_moves(MoveView M, const uint32_t *node, uint32_t count,
                                                       const uint32_t *inc_off, const uint32_t *inc,
                                                       const uint32_t *pins, const int32_t *nwgt, uint32_t k,
                                                       int32_t *omega, int64_t *gain) {
    const uint32_t lane = __lane_id();
    for (uint32_t b0 = blockIdx.x * BLOCK; b0 < count; b0 += gridDim.x * BLOCK) {
        const uint32_t i = b0 + threadIdx.x;
        uint32_t u = 0, s = 0, t = 0, j0 = 0, j1 = 0, iu;
        const bool act = i < count && M.from[i] != NONE && M.moved(node[i], &iu);
        if (act) {
            u = node[i]; s = M.from[i]; t = M.target[i];
            j0 = inc_off[u]; j1 = inc_off[u + 1];
        }
        const bool wide = act && j1 - j0 > 32;
        int64_t g = 0;
        if (act && !wide)
            for (uint32_t j = j0; j < j1; ++j) graph_edge(M, i, u, s, t, inc[j], pins, nwgt, k, omega, &g);
        if (gain && i < count && !wide) gain[i] = g;
        uint64_t wm = __ballot(wide);
        while (wm) {  // the wave takes its wide moves one at a time
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t hi_ = __shfl(i, h, WAVE), hu = __shfl(u, h, WAVE), hs = __shfl(s, h, WAVE),
                           ht = __shfl(t, h, WAVE), hj0 = __shfl(j0, h, WAVE), hj1 = __shfl(j1, h, WAVE);
            int64_t hg = 0;
            for (uint32_t j = hj0 + lane; j < hj1; j += WAVE)
                graph_edge(M, hi_, hu, hs, ht, inc[j], pins, nwgt, k, omega, &hg);
            hg = wave_sum(hg);
            if (gain && (int)lane == h) gain[hi_] = hg;
        }
    }
}

struct GtBufs {
    uint64_t *lam, *lam1;
    uint32_t *idx, *from, *stamp, *longl, *scal;
};

void plan_table(Arena &A, uint32_t m, uint32_t k, GtBufs &B) {
    const size_t kw = (k + 63) / 64;
    B.lam = A.alloc<uint64_t>((size_t)m * kw);
    B.lam1 = A.alloc<uint64_t>((size_t)m * kw);
    B.longl = A.alloc<uint32_t>(m);
    B.scal = A.alloc<uint32_t>(64);
}

void plan_moves(Arena &A, uint32_t n, uint32_t m, uint32_t count, GtBufs &B) {
    B.idx = A.alloc<uint32_t>(n);
    B.from = A.alloc<uint32_t>(count);
    B.stamp = A.alloc<uint32_t>(m);
    B.longl = A.alloc<uint32_t>(m);
    B.scal = A.alloc<uint32_t>(64);
}

template <int KW>
void table_t(const hgp_hg &h, uint32_t k, const uint32_t *part, int32_t *ben, int32_t *pen, Arena &A,
             hipStream_t st) {
    size_t mk = A.mark();
    GtBufs B{};
    plan_table(A, h.m, k, B);
    if (A.measure) { A.release(mk); return; }
    uint32_t *nlong = B.scal;
    fill<uint32_t>(B.scal, 64, 0u, st);
    if (h.m) {
        k_gt_conn<KW><<<grid_for(h.m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, h.m, part, B.lam,
                                                                           B.lam1, B.longl, nlong);
        HGP_LAUNCH_CHECK();
        k_gt_conn_long<KW><<<FILL_BLOCKS / 4, BLOCK, 0, st>>>(h.pin_off, h.pins, B.longl, nlong, part, B.lam,
                                                              B.lam1);
        HGP_LAUNCH_CHECK();
    }
    // about eight waves per CU, each over a contiguous range of vertices
    const unsigned blocks = (unsigned)std::min<size_t>(2 * FILL_BLOCKS, ((size_t)h.n + 63) / 64);
    k_gt_rows<KW><<<blocks, BLOCK, 0, st>>>(h.inc_off, h.inc, h.nwgt, part, B.lam, B.lam1, h.n, k, ben, pen);
    HGP_LAUNCH_CHECK();
    A.release(mk);
}

// Marks the moves and checks them; returns false on invalid moves.  Syncs.
bool mark_moves(const hgp_hg &h, uint32_t k, const uint32_t *part, const uint32_t *node, const uint32_t *target,
                uint32_t count, const GtBufs &B, hipStream_t st) {
    fill<uint32_t>(B.idx, h.n, NONE, st);
    fill<uint32_t>(B.stamp, h.m, 0u, st);
    fill<uint32_t>(B.scal, 64, 0u, st);
    k_gt_mark<<<grid_for(count, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(node, target, count, h.n, k, part, B.idx,
                                                                     B.from, B.scal + 1);
    HGP_LAUNCH_CHECK();
    uint32_t err = 0;
    HGP_CHECK_HIP(hipMemcpyAsync(&err, B.scal + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    stream_sync(st);
    return err == 0;
}

}  // namespace

size_t gaintable_workspace(uint32_t n, uint32_t m, uint32_t k, uint32_t count) {
    Arena A(nullptr, 0);
    GtBufs B{};
    plan_table(A, m, k, B);
    size_t a = A.peak;
    Arena C(nullptr, 0);
    plan_moves(C, n, m, count, B);
    return a > C.peak ? a : C.peak;
}

void gain_table(const hgp_hg &h, uint32_t k, const uint32_t *part, int32_t *ben, int32_t *pen, Arena &A,
                hipStream_t st) {
    switch ((k + 63) / 64) {
        case 1: table_t<1>(h, k, part, ben, pen, A, st); break;
        case 2: table_t<2>(h, k, part, ben, pen, A, st); break;
        case 3: table_t<3>(h, k, part, ben, pen, A, st); break;
        default: table_t<4>(h, k, part, ben, pen, A, st); break;
    }
}

hgp_status gain_table_update(const hgp_hg &h, uint32_t k, uint32_t *part, const uint32_t *node,
                             const uint32_t *target, uint32_t count, int32_t *ben, int32_t *pen, Arena &A,
                             hipStream_t st) {
    size_t mk = A.mark();
    GtBufs B{};
    plan_moves(A, h.n, h.m, count, B);
    if (A.measure || count == 0) { A.release(mk); return HGP_OK; }
    if (!mark_moves(h, k, part, node, target, count, B, st)) { A.release(mk); return HGP_E_INVALID; }
    const MoveView M{B.idx, target, B.from, part};
    uint32_t *nlong = B.scal;
    const unsigned g = grid_for(count, BLOCK, FILL_BLOCKS);
    k_gt_nets<OP_UPDATE><<<g, BLOCK, 0, st>>>(M, node, count, h.inc_off, h.inc, h.pin_off, h.pins, h.nwgt, k,
                                              B.stamp, 1u, B.longl, nlong, ben, pen, nullptr);
    HGP_LAUNCH_CHECK();
    k_gt_long<OP_UPDATE><<<FILL_BLOCKS / 4, BLOCK, 0, st>>>(M, B.longl, nlong, h.pin_off, h.pins, h.nwgt, k, ben,
                                                            pen, nullptr);
    HGP_LAUNCH_CHECK();
    k_gt_mover_benefit<<<g, BLOCK, 0, st>>>(M, node, count, h.inc_off, h.inc, h.pin_off, h.pins, h.nwgt, ben);
    HGP_LAUNCH_CHECK();
    k_gt_apply<<<g, BLOCK, 0, st>>>(M, node, count, part);
    HGP_LAUNCH_CHECK();
    stream_sync(st);
    A.release(mk);
    return HGP_OK;
}

hgp_status gain_recalc(const hgp_hg &h, uint32_t k, const uint32_t *part, const uint32_t *node,
                       const uint32_t *target, uint32_t count, int64_t *gain, Arena &A, hipStream_t st) {
    size_t mk = A.mark();
    GtBufs B{};
    plan_moves(A, h.n, h.m, count, B);
    if (A.measure || count == 0) { A.release(mk); return HGP_OK; }
    if (!mark_moves(h, k, part, node, target, count, B, st)) { A.release(mk); return HGP_E_INVALID; }
    const MoveView M{B.idx, target, B.from, part};
    uint32_t *nlong = B.scal;
    HGP_CHECK_HIP(hipMemsetAsync(gain, 0, sizeof(int64_t) * count, st));
    const unsigned g = grid_for(count, BLOCK, FILL_BLOCKS);
    k_gt_nets<OP_RECALC><<<g, BLOCK, 0, st>>>(M, node, count, h.inc_off, h.inc, h.pin_off, h.pins, h.nwgt, k,
                                              B.stamp, 1u, B.longl, nlong, nullptr, nullptr,
                                              (unsigned long long *)gain);
    HGP_LAUNCH_CHECK();
    k_gt_long<OP_RECALC><<<FILL_BLOCKS / 4, BLOCK, 0, st>>>(M, B.longl, nlong, h.pin_off, h.pins, h.nwgt, k,
                                                            nullptr, nullptr, (unsigned long long *)gain);
    HGP_LAUNCH_CHECK();
    stream_sync(st);
    A.release(mk);
    return HGP_OK;
}


// A graph: p = 2m and no net of other than two pins (one device read-back).
static bool is_graph(const hgp_hg &h, const GtBufs &B, hipStream_t st) {
    if ((uint64_t)h.p != 2ull * h.m) return false;
    if (h.m == 0) return true;
    fill<uint32_t>(B.scal + 2, 1, 0u, st);
    k_non_edges<<<grid_for(h.m, BLOCK, REDUCE_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.m, B.scal + 2);
    HGP_LAUNCH_CHECK();
    uint32_t bad = 0;
    HGP_CHECK_HIP(hipMemcpyAsync(&bad, B.scal + 2, sizeof(bad), hipMemcpyDeviceToHost, st));
    stream_sync(st);
    return bad == 0;
}

template <int KW>
static void graph_rows_t(const hgp_hg &h, uint32_t k, const uint32_t *part, int32_t *omega, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<size_t>(2 * FILL_BLOCKS, ((size_t)h.n + 63) / 64);
    k_ggt_rows<KW><<<blocks, BLOCK, 0, st>>>(h.inc_off, h.inc, h.pins, h.nwgt, part, h.n, k, omega);
    HGP_LAUNCH_CHECK();
}

hgp_status graph_gain_table(const hgp_hg &h, uint32_t k, const uint32_t *part, int32_t *omega, Arena &A,
                            hipStream_t st) {
    size_t mk = A.mark();
    GtBufs B{};
    plan_moves(A, h.n, h.m, 0, B);
    if (A.measure) { A.release(mk); return HGP_OK; }
    if (!is_graph(h, B, st)) { A.release(mk); return HGP_E_INVALID; }
    if (h.n) {
        switch ((k + 63) / 64) {
            case 1: graph_rows_t<1>(h, k, part, omega, st); break;
            case 2: graph_rows_t<2>(h, k, part, omega, st); break;
            case 3: graph_rows_t<3>(h, k, part, omega, st); break;
            default: graph_rows_t<4>(h, k, part, omega, st); break;
        }
    }
    A.release(mk);
    return HGP_OK;
}

hgp_status graph_moves(const hgp_hg &h, uint32_t k, uint32_t *part, const uint32_t *node, const uint32_t *target,
                       uint32_t count, int32_t *omega, int64_t *gain, Arena &A, hipStream_t st) {
    size_t mk = A.mark();
    GtBufs B{};
    plan_moves(A, h.n, h.m, count, B);
    if (A.measure) { A.release(mk); return HGP_OK; }
    if (!is_graph(h, B, st)) { A.release(mk); return HGP_E_INVALID; }
    if (count == 0) { A.release(mk); return HGP_OK; }
    if (!mark_moves(h, k, part, node, target, count, B, st)) { A.release(mk); return HGP_E_INVALID; }
    const MoveView M{B.idx, target, B.from, part};
    const unsigned g = grid_for(count, BLOCK, FILL_BLOCKS);
    k_graph_moves<<<g, BLOCK, 0, st>>>(M, node, count, h.inc_off, h.inc, h.pins, h.nwgt, k, omega, gain);
    HGP_LAUNCH_CHECK();
    k_gt_apply<<<g, BLOCK, 0, st>>>(M, node, count, part);
    HGP_LAUNCH_CHECK();
    stream_sync(st);
    A.release(mk);
    return HGP_OK;
}

}  // namespace hgp
