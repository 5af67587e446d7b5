// Community detection for community-aware coarsening (paper Sec. 4.3): the
// Louvain method on the bipartite graph representation of the hypergraph,
// made deterministic as in Sec. 11 (synchronous local moving in sub-rounds).
//
//  - G_x: node u < n is vertex u, node n + e is net e, one edge {u, n + e}
//    per pin (edge j = pin position j) of weight w(e).  It is stored as a
//    two-pin hypergraph, so the contraction of Sec. 4.2 builds the Louvain
//    levels (self-loops dropped, parallel edges merged, node weights -- the
//    volumes -- summed).
//  - A sub-round aggregates w(x, C) for its nodes by sorting (node rank,
//    neighbour community) keys with the device radix sort; a lane per node
//    (a wave for more than 64 edges) then walks the node's sorted run of
//    communities and scores each one exactly in int64: score(C) = m2 w(x, C)
//    - vol(x) vol(C) against score(A) = m2 w(x, A) - vol(x) (vol(A) - vol(x)),
//    the modularity gain times m2^2 / 2.  All moves of a sub-round are
//    applied together; the community volumes are integers, so their atomic
//    updates give the same sums in any order.
#include "kernels.h"
#include "prims.h"

#include <algorithm>

namespace hgp {

namespace {

constexpr uint32_t LV_ROUNDS = 5;     // local-moving rounds per level at most
constexpr uint32_t LV_SUBROUNDS = 5;  // sub-rounds per round
constexpr uint32_t LV_LEVELS = 16;    // Louvain levels at most
constexpr uint32_t LV_WIDE = 32;      // lists longer than this: a wave each
constexpr uint32_t LV_SEG = 64;       // sorted runs longer than this: a wave each
constexpr uint32_t LV_DIRECT = 16;    // nodes of at most this many edges decide without the sort
constexpr uint32_t LV_WAVE = 512;     // up to this many: a wave and an LDS table per node (k_lv_wave)
constexpr uint32_t LV_TBL = 1024;     // its slots (power of two, at least 2 LV_WAVE)

// --- the bipartite graph ----------------------------------------------------

// Sum over nets of |e| w(e) (half the total volume), spread accumulator.
__global__ __launch_bounds__(BLOCK) void k_bip_volume(const uint32_t *pin_off, const int32_t *nwgt, uint32_t m,
                                                      int64_t *acc) {
    int64_t v = 0;
    for (uint32_t e = blockIdx.x * BLOCK + threadIdx.x; e < m; e += gridDim.x * BLOCK)
        v += (int64_t)(pin_off[e + 1] - pin_off[e]) * nwgt[e];
    v = wave_sum(v);
    __shared__ int64_t red[BLOCK / WAVE];
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BLOCK / WAVE; ++q) v += red[q];
        if (v) spread_add_i64(acc, v);
    }
}

__global__ void k_total(const int64_t *acc, int64_t *out) {
    const int64_t t = spread_total_wave(acc);
    if (threadIdx.x == 0) *out = t;
}

// Net nodes and the edge list: a thread per net of up to LV_WIDE pins, the
// wave for a longer one.  Edge j = {pins[j], n + e}: xpins[2j], xpins[2j+1];
// the net node lists its edges pin_off[e] .. pin_off[e+1]-1 at p + j.
__global__ __launch_bounds__(BLOCK) void k_bip_nets(const uint32_t *pin_off, const uint32_t *pins,
                                                    const int32_t *nwgt, uint32_t n, uint32_t m, uint32_t p,
                                                    uint32_t *xpin_off, uint32_t *xpins, uint32_t *xinc_off,
                                                    uint32_t *xinc, int32_t *xvw, int32_t *xnw) {
    for (uint32_t e0 = blockIdx.x * BLOCK; e0 < m; e0 += gridDim.x * BLOCK) {
        const uint32_t e = e0 + threadIdx.x;
        uint32_t b = 0, sz = 0;
        int32_t w = 0;
        if (e < m) {
            b = pin_off[e];
            sz = pin_off[e + 1] - b;
            w = nwgt[e];
            xinc_off[n + e + 1] = p + b + sz;
            xvw[n + e] = (int32_t)((int64_t)sz * w);
        }
        const bool wide = sz > LV_WIDE;
        if (e < m && !wide)
            for (uint32_t j = b; j < b + sz; ++j) {
                xpin_off[j] = 2 * j;
                xpins[2 * (size_t)j] = pins[j];
                xpins[2 * (size_t)j + 1] = n + e;
                xnw[j] = w;
                xinc[(size_t)p + j] = j;
            }
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t he = __shfl(e, h, WAVE), hb = __shfl(b, h, WAVE), hs = __shfl(sz, h, WAVE);
            const int32_t hw = __shfl(w, h, WAVE);
            for (uint32_t j = hb + __lane_id(); j < hb + hs; j += WAVE) {
                xpin_off[j] = 2 * j;
                xpins[2 * (size_t)j] = pins[j];
                xpins[2 * (size_t)j + 1] = n + he;
                xnw[j] = hw;
                xinc[(size_t)p + j] = j;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        xpin_off[p] = 2 * p;
        xinc_off[n] = p;
    }
}

// Position of u among the (ascending) pins of the net starting at b.
__device__ inline uint32_t pin_pos(const uint32_t *pins, uint32_t b, uint32_t sz, uint32_t u) {
    uint32_t lo = 0, hi = sz;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pins[b + mid] < u) lo = mid + 1; else hi = mid;
    }
    return b + lo;
}

// Vertex nodes: the edges of u in the order of its nets (the edge of net e
// is u's pin position in e), and vol(u) = the weight of its nets.  A thread
// per vertex of up to LV_WIDE nets, the wave for a larger one.
__global__ __launch_bounds__(BLOCK) void k_bip_vertices(const uint32_t *inc_off, const uint32_t *inc,
                                                        const uint32_t *pin_off, const uint32_t *pins,
                                                        const int32_t *nwgt, uint32_t n, uint32_t *xinc_off,
                                                        uint32_t *xinc, int32_t *xvw) {
    for (uint32_t u0 = blockIdx.x * BLOCK; u0 < n; u0 += gridDim.x * BLOCK) {
        const uint32_t u = u0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (u < n) {
            j0 = inc_off[u];
            j1 = inc_off[u + 1];
            xinc_off[u] = j0;
        }
        const bool wide = j1 - j0 > LV_WIDE;
        if (u < n && !wide) {
            int64_t vol = 0;
            for (uint32_t j = j0; j < j1; ++j) {
                const uint32_t e = inc[j], b = pin_off[e];
                xinc[j] = pin_pos(pins, b, pin_off[e + 1] - b, u);
                vol += nwgt[e];
            }
            xvw[u] = (int32_t)vol;
        }
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t hu = __shfl(u, h, WAVE), hj0 = __shfl(j0, h, WAVE), hj1 = __shfl(j1, h, WAVE);
            int64_t vol = 0;
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) {
                const uint32_t e = inc[j], b = pin_off[e];
                xinc[j] = pin_pos(pins, b, pin_off[e + 1] - b, hu);
                vol += nwgt[e];
            }
            vol = wave_sum(vol);
            if ((int)__lane_id() == h) xvw[hu] = (int32_t)vol;
        }
    }
}

// --- local moving -------------------------------------------------------------

__global__ void k_lv_init(const int32_t *vw, uint32_t N, uint32_t *comm, int64_t *cvol) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < N; x += gridDim.x * blockDim.x) {
        comm[x] = x;
        cvol[x] = vw[x];
    }
}

// Nodes of sub-round (r, s), numbered in ID order, with the offsets of the
// edges that go through the sort: the scan value is (1 << 32 | degree) for a
// node of the sub-round with more than LV_WAVE edges, (1 << 32) for the
// others (they decide from their own edges, k_lv_direct and k_lv_wave).
struct SelPack {
    const uint32_t *inc_off;
    uint64_t mseed;
    uint32_t level, r, s;
    __device__ uint64_t operator()(size_t x) const {
        if (tag_hash(mseed, 4, level, r, (uint32_t)x) % LV_SUBROUNDS != s) return 0ull;
        const uint32_t d = inc_off[x + 1] - inc_off[x];
        return (1ull << 32) | (uint64_t)(d > LV_WAVE ? d : 0u);
    }
};
struct SelStore {
    uint32_t *list, *ioff;
    __device__ void operator()(size_t x, uint64_t excl, uint64_t v) const {
        if (v) {
            list[excl >> 32] = (uint32_t)x;
            ioff[excl >> 32] = (uint32_t)excl;
        }
    }
};

// Decision of every node of the sub-round with at most LV_DIRECT edges, from
// its own edges: the (community, weight) pair of each edge goes into the
// thread's column of an LDS table in community order (insertion), and the
// runs are walked as k_lv_decide walks a sorted run.  Same scores, same
// ties, no keys written and no sort.
__global__ __launch_bounds__(BLOCK) void k_lv_direct(const uint32_t *list, uint32_t count, const uint32_t *inc_off,
                                                     const uint32_t *inc, const uint32_t *pin_off,
                                                     const uint32_t *pins, const int32_t *nwgt,
                                                     const uint32_t *comm, const int64_t *cvol, const int32_t *vw,
                                                     int64_t m2, uint32_t *dec, uint32_t *mid, uint32_t *nmid);

// Keys (rank of the node in the sub-round, community of the neighbour) and
// the edge weights, at the node's offset (nodes of more than LV_WAVE edges
// only).
__global__ __launch_bounds__(BLOCK) void k_lv_emit(const uint32_t *list, const uint32_t *ioff, uint32_t count,
                                                   const uint32_t *inc_off, const uint32_t *inc,
                                                   const uint32_t *pin_off, const uint32_t *pins,
                                                   const int32_t *nwgt, const uint32_t *comm, int cb,
                                                   uint64_t *keys, uint32_t *vals) {
    for (uint32_t i0 = blockIdx.x * BLOCK; i0 < count; i0 += gridDim.x * BLOCK) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t x = 0, j0 = 0, j1 = 0, o = 0;
        if (i < count) {
            x = list[i];
            j0 = inc_off[x];
            j1 = inc_off[x + 1];
            o = ioff[i];
        }
        if (j1 - j0 <= LV_WAVE) j1 = j0;  // decided by k_lv_direct or k_lv_wave: nothing to emit
        const bool wide = j1 - j0 > LV_WIDE;
        auto edge = [&](uint32_t xi, uint32_t xx, uint32_t j, uint32_t at) {
            const uint32_t e = inc[j];
            const uint2 ab = *(const uint2 *)(pins + 2 * (size_t)e);  // two pins at 2e (see k_lv_direct)
            const uint32_t a = ab.x, c = ab.y;
            keys[at] = ((uint64_t)xi << cb) | comm[a == xx ? c : a];
            vals[at] = (uint32_t)nwgt[e];
        };
        if (i < count && !wide)
            for (uint32_t j = j0; j < j1; ++j) edge(i, x, j, o + (j - j0));
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t hi = __shfl(i, h, WAVE), hx = __shfl(x, h, WAVE), hj0 = __shfl(j0, h, WAVE),
                           hj1 = __shfl(j1, h, WAVE), ho = __shfl(o, h, WAVE);
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) edge(hi, hx, j, ho + (j - hj0));
        }
    }
}

// Best community of a node from its sorted (community, weight) run.
struct Best {
    int64_t score;
    uint32_t c;
};
__device__ inline void best_merge(Best &b, int64_t s, uint32_t c) {
    if (c == NONE) return;
    if (b.c == NONE || s > b.score || (s == b.score && c < b.c)) { b.score = s; b.c = c; }
}

// Decision of every node of the sub-round with more than LV_WAVE edges
// (dec[i] = the community it moves to, or NONE; the others have an empty
// run and are left to k_lv_direct and k_lv_wave).  A lane walks a run of up to LV_SEG
// entries; a wave takes a longer run 64 entries at a time (segmented sum of
// equal communities, the open group's sum carried into the next step).
__global__ __launch_bounds__(BLOCK) void k_lv_decide(const uint32_t *list, const uint32_t *ioff, uint32_t count,
                                                     const uint64_t *keys, const uint32_t *vals,
                                                     const uint32_t *comm, const int64_t *cvol, const int32_t *vw,
                                                     int64_t m2, uint64_t cmask, uint32_t *dec) {
    const uint32_t lane = __lane_id();
    for (uint32_t i0 = blockIdx.x * BLOCK; i0 < count; i0 += gridDim.x * BLOCK) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t b = 0, e = 0, x = 0, A = 0;
        int64_t vx = 0;
        if (i < count) {
            b = ioff[i];
            e = ioff[i + 1];
            x = list[i];
            A = comm[x];
            vx = vw[x];
        }
        const bool wide = e - b > LV_SEG;
        if (i < count && !wide && e > b) {
            Best best{0, NONE};
            int64_t wA = 0, acc = 0;
            uint32_t cur = NONE;
            for (uint32_t q = b; q <= e; ++q) {
                const uint32_t c = q < e ? (uint32_t)(keys[q] & cmask) : NONE;
                if (c != cur) {
                    if (cur != NONE) {
                        if (cur == A) wA = acc;
                        else best_merge(best, m2 * acc - vx * cvol[cur], cur);
                    }
                    cur = c;
                    acc = 0;
                }
                if (q < e) acc += vals[q];
            }
            const int64_t sA = m2 * wA - vx * (cvol[A] - vx);
            dec[i] = (best.c != NONE && best.score > sA) ? best.c : NONE;
        }
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t hi = __shfl(i, h, WAVE), hb = __shfl(b, h, WAVE), he = __shfl(e, h, WAVE),
                           hA = __shfl(A, h, WAVE);
            const int64_t hvx = __shfl(vx, h, WAVE);
            Best best{0, NONE};
            int64_t wA = 0, carry = 0;
            for (uint32_t c0 = hb; c0 < he; c0 += WAVE) {
                const uint32_t q = c0 + lane;
                const bool valid = q < he;
                uint32_t c = NONE;
                int64_t v = 0;
                bool head = true, tail = false;
                if (valid) {
                    c = (uint32_t)(keys[q] & cmask);
                    v = vals[q];
                    head = q == hb || (uint32_t)(keys[q - 1] & cmask) != c;
                    tail = q + 1 == he || (uint32_t)(keys[q + 1] & cmask) != c;
                }
                // segmented inclusive sum; f: a group start at or before the lane
                bool f = head;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    const int64_t t = __shfl_up(v, o, WAVE);
                    const bool tf = __shfl_up((int)f, o, WAVE) != 0;
                    if (lane >= (uint32_t)o && !f) v += t;
                    if (lane >= (uint32_t)o) f = f || tf;
                }
                if (!f) v += carry;  // the group open at the end of the previous step
                Best mine{0, NONE};
                int64_t a_part = 0;
                if (valid && tail) {
                    if (c == hA) a_part = v;
                    else best_merge(mine, m2 * v - hvx * cvol[c], c);
                }
                wA += wave_sum(a_part);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const int64_t os = __shfl_xor(mine.score, o, WAVE);
                    const uint32_t oc = __shfl_xor(mine.c, o, WAVE);
                    best_merge(mine, os, oc);
                }
                best_merge(best, mine.score, mine.c);
                // the last lane's group continues into the next step unless it ends here
                const uint32_t last = (he - c0 < WAVE ? he - c0 : WAVE) - 1;
                const bool open = !__shfl((int)tail, (int)last, WAVE);
                carry = open ? __shfl(v, (int)last, WAVE) : 0;
            }
            if ((int)lane == h) {
                const int64_t sA = m2 * wA - hvx * (cvol[hA] - hvx);
                dec[hi] = (best.c != NONE && best.score > sA) ? best.c : NONE;
            }
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_lv_direct(const uint32_t *list, uint32_t count, const uint32_t *inc_off,
                                                     const uint32_t *inc, const uint32_t *pin_off,
                                                     const uint32_t *pins, const int32_t *nwgt,
                                                     const uint32_t *comm, const int64_t *cvol, const int32_t *vw,
                                                     int64_t m2, uint32_t *dec, uint32_t *mid, uint32_t *nmid) {
    __shared__ uint32_t sc[LV_DIRECT][BLOCK];  // column per thread: no bank conflicts
    __shared__ int32_t sw[LV_DIRECT][BLOCK];
    const uint32_t t = threadIdx.x;
    for (uint32_t i0 = blockIdx.x * BLOCK; i0 < count; i0 += gridDim.x * BLOCK) {  // uniform per block
        const uint32_t i = i0 + t;
        uint32_t x = 0, j0 = 0, deg = 0;
        if (i < count) {
            x = list[i];
            j0 = inc_off[x];
            deg = inc_off[x + 1] - j0;
        }
        // nodes of up to LV_WAVE edges are listed for k_lv_wave, longer ones go through the sort
        const uint32_t at = warp_agg_append(nmid, i < count && deg > LV_DIRECT && deg <= LV_WAVE);
        if (i < count && deg > LV_DIRECT && deg <= LV_WAVE) mid[at] = i;
        if (i >= count || deg > LV_DIRECT) continue;
        // eight edges at a time: every load of a stage is issued before any
        // is used (edge, its offsets, its endpoints, the neighbour's
        // community), then each pair is inserted in community order
        for (uint32_t q0 = 0; q0 < deg; q0 += 8) {
            uint32_t e[8], b[8], c[8];
            int32_t w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) e[k] = q0 + k < deg ? inc[j0 + q0 + k] : NONE;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // every edge of the bipartite graph and of its contractions
                // has two pins, at 2e and 2e + 1: one 8-byte load
                const uint2 ab = e[k] != NONE ? *(const uint2 *)(pins + 2 * (size_t)e[k]) : make_uint2(0u, 0u);
                b[k] = ab.x == x ? ab.y : ab.x;  // the neighbour
                w[k] = e[k] != NONE ? nwgt[e[k]] : 0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) c[k] = b[k];
#pragma unroll
            for (int k = 0; k < 8; ++k) c[k] = e[k] != NONE ? comm[c[k]] : NONE;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (e[k] == NONE) continue;
                uint32_t z = q0 + k;
                while (z > 0 && sc[z - 1][t] > c[k]) {
                    sc[z][t] = sc[z - 1][t];
                    sw[z][t] = sw[z - 1][t];
                    --z;
                }
                sc[z][t] = c[k];
                sw[z][t] = w[k];
            }
        }
        const uint32_t A = comm[x];
        const int64_t vx = vw[x];
        Best best{0, NONE};
        int64_t wA = 0, acc = 0;
        uint32_t cur = NONE;
        for (uint32_t q = 0; q <= deg; ++q) {
            const uint32_t c = q < deg ? sc[q][t] : NONE;
            if (c != cur) {
                if (cur != NONE) {
                    if (cur == A) wA = acc;
                    else best_merge(best, m2 * acc - vx * cvol[cur], cur);
                }
                cur = c;
                acc = 0;
            }
            if (q < deg) acc += sw[q][t];
        }
        const int64_t sA = m2 * wA - vx * (cvol[A] - vx);
        dec[i] = (best.c != NONE && best.score > sA) ? best.c : NONE;
    }
}

// Decision of the listed nodes of LV_DIRECT + 1 .. LV_WAVE edges: a wave per
// node sums the weight of each neighbour community in an LDS hash table
// (linear probing, at most LV_WAVE distinct keys in LV_TBL slots), then
// every lane judges its slots and the wave keeps the best (largest score,
// then the smaller community), as the sorted path does over its runs.
constexpr int LVW_WAVES = BLOCK / WAVE;
__global__ __launch_bounds__(BLOCK) void k_lv_wave(const uint32_t *list, const uint32_t *mid, const uint32_t *nmid,
                                                   const uint32_t *inc_off, const uint32_t *inc,
                                                   const uint32_t *pins, const int32_t *nwgt, const uint32_t *comm,
                                                   const int64_t *cvol, const int32_t *vw, int64_t m2,
                                                   uint32_t *dec) {
    __shared__ uint32_t tk[LVW_WAVES][LV_TBL];
    __shared__ unsigned long long tw[LVW_WAVES][LV_TBL];
    const uint32_t w = threadIdx.x / WAVE, lane = __lane_id();
    uint32_t *K = tk[w];
    unsigned long long *V = tw[w];
    const uint32_t cnt = *nmid;
    for (uint32_t q = blockIdx.x * LVW_WAVES + w; q < cnt; q += gridDim.x * LVW_WAVES) {  // uniform per wave
        const uint32_t i = mid[q], x = list[i], j0 = inc_off[x], j1 = inc_off[x + 1];
        for (uint32_t z = lane; z < LV_TBL; z += WAVE) {
            K[z] = NONE;
            V[z] = 0ull;
        }
        wave_sync();
        for (uint32_t j = j0 + lane; j < j1; j += WAVE) {
            const uint32_t e = inc[j];
            const uint2 ab = *(const uint2 *)(pins + 2 * (size_t)e);  // two pins at 2e
            const uint32_t c = comm[ab.x == x ? ab.y : ab.x];
            uint32_t z = (c * 0x9E3779B1u) >> (32 - 10);
            static_assert(LV_TBL == 1024, "the slot hash takes 10 bits");
            for (;;) {
                const uint32_t old = atomicCAS(&K[z], NONE, c);
                if (old == NONE || old == c) break;
                z = (z + 1) & (LV_TBL - 1);
            }
            atomicAdd(&V[z], (unsigned long long)(int64_t)nwgt[e]);
        }
        wave_sync();
        const uint32_t A = comm[x];
        const int64_t vx = vw[x];
        Best best{0, NONE};
        int64_t wA = 0;
        for (uint32_t z = lane; z < LV_TBL; z += WAVE) {
            const uint32_t c = K[z];
            if (c == NONE) continue;
            const int64_t acc = (int64_t)V[z];
            if (c == A) wA = acc;
            else best_merge(best, m2 * acc - vx * cvol[c], c);
        }
        wA = wave_sum(wA);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int64_t os = __shfl_xor(best.score, o, WAVE);
            const uint32_t oc = __shfl_xor(best.c, o, WAVE);
            best_merge(best, os, oc);
        }
        if (lane == 0) {
            const int64_t sA = m2 * wA - vx * (cvol[A] - vx);
            dec[i] = (best.c != NONE && best.score > sA) ? best.c : NONE;
        }
        wave_sync();  // the table is read before the next node clears it
    }
}

// All moves of the sub-round; the moves are counted per block into a spread
// accumulator.
__global__ __launch_bounds__(BLOCK) void k_lv_apply(const uint32_t *list, const uint32_t *dec, uint32_t count,
                                                    const int32_t *vw, uint32_t *comm, int64_t *cvol,
                                                    int64_t *moves) {
    int64_t mv = 0;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        const uint32_t C = dec[i];
        if (C == NONE) continue;
        const uint32_t x = list[i];
        const int64_t v = vw[x];
        atomic_add_i64(&cvol[comm[x]], -v);
        atomic_add_i64(&cvol[C], v);
        comm[x] = C;
        ++mv;
    }
    mv = wave_sum(mv);
    __shared__ int64_t red[BLOCK / WAVE];
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = mv;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BLOCK / WAVE; ++q) mv += red[q];
        if (mv) spread_add_i64(moves, mv);
    }
}

// Representative of every community: its smallest node.
__global__ void k_lv_minid(const uint32_t *comm, uint32_t N, uint32_t *minid) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < N; x += gridDim.x * blockDim.x)
        atomicMin(&minid[comm[x]], x);
}
__global__ void k_lv_rep(const uint32_t *comm, const uint32_t *minid, uint32_t N, uint32_t *rep) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < N; x += gridDim.x * blockDim.x)
        rep[x] = minid[comm[x]];
}
__global__ void k_lv_map(const uint32_t *cid, uint32_t n, uint32_t *node) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
        node[u] = cid[node[u]];
}

struct LvGraph {
    uint32_t *pin_off, *pins, *inc_off, *inc;
    int32_t *vwgt, *nwgt;
};

struct LvBufs {
    LvGraph G[2];
    uint32_t *comm, *rep, *cid, *minid, *node, *list, *ioff, *dec, *mid, *nmid;
    int64_t *cvol, *acc, *tot;
};

void plan(Arena &A, uint32_t n, uint32_t m, uint32_t p, LvBufs &B) {
    const size_t N = (size_t)n + m;
    for (int b = 0; b < 2; ++b) {
        B.G[b].pin_off = A.alloc<uint32_t>((size_t)p + 1);
        B.G[b].pins = A.alloc<uint32_t>(2 * (size_t)p);
        B.G[b].inc_off = A.alloc<uint32_t>(N + 1);
        B.G[b].inc = A.alloc<uint32_t>(2 * (size_t)p);
        B.G[b].vwgt = A.alloc<int32_t>(N);
        B.G[b].nwgt = A.alloc<int32_t>(p);
    }
    B.comm = A.alloc<uint32_t>(N);
    B.rep = A.alloc<uint32_t>(N);
    B.cid = A.alloc<uint32_t>(N);
    B.minid = A.alloc<uint32_t>(N);
    B.node = A.alloc<uint32_t>(n);
    B.list = A.alloc<uint32_t>(N);
    B.ioff = A.alloc<uint32_t>(N + 1);
    B.dec = A.alloc<uint32_t>(N);
    B.mid = A.alloc<uint32_t>(N);
    B.nmid = A.alloc<uint32_t>(1);
    B.cvol = A.alloc<int64_t>(N);
    B.acc = A.alloc<int64_t>((size_t)SPREAD * SPREAD_I64 * (LV_ROUNDS + 1));
    B.tot = A.alloc<int64_t>(LV_ROUNDS + 1);
}

// Sub-round temporaries: the keys and weights of at most every edge end (2p)
// and the sort's alternate buffers, or the contraction's scratch.
size_t temp_bytes(uint32_t n, uint32_t m, uint32_t p) {
    Arena A(nullptr, 0);
    const size_t items = 2 * (size_t)p;
    A.alloc<uint64_t>(items);
    A.alloc<uint32_t>(items);
    A.alloc<uint64_t>(items);
    A.alloc<uint32_t>(items);
    sort_reserve(A, items);
    scan_reserve<uint64_t>(A, (size_t)n + m);
    A.alloc<uint64_t>(4);
    const size_t a = A.peak;
    const size_t c = contract_workspace(n + m, p, 2 * p);
    return std::max(a, c);
}

__global__ void k_comm_down(uint32_t n, const uint32_t *cid, const uint32_t *comm, uint32_t *ccomm) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
        ccomm[cid[u]] = comm[u];  // every member of a cluster has its community
}

}  // namespace

void community_down(uint32_t n, const uint32_t *cid, const uint32_t *comm, uint32_t *ccomm, hipStream_t st) {
    k_comm_down<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(n, cid, comm, ccomm);
    HGP_LAUNCH_CHECK();
}

size_t community_workspace(uint32_t n, uint32_t m, uint32_t p) {
    Arena A(nullptr, 0);
    LvBufs B;
    plan(A, n, m, p, B);
    return A.peak + temp_bytes(n, m, p) + 4096;
}

hgp_status communities(const hgp_hg &h, uint64_t seed, uint32_t *comm_out, uint32_t *levels_out, Arena &A,
                       hipStream_t st) {
    const uint32_t n = h.n, m = h.m, p = h.p;
    if ((uint64_t)n + m >= 0xFFFFFFFFull || (uint64_t)p >= (1ull << 31)) return HGP_E_UNSUPPORTED;
    size_t mk = A.mark();
    LvBufs B;
    plan(A, n, m, p, B);
    const size_t tmk = A.mark();
    if (A.measure) { A.release(mk); return HGP_OK; }
    const uint32_t N = n + m;
    // total volume 2 * sum |e| w(e): below 2^31, so that the node weights and
    // every product of two volumes fit
    HGP_CHECK_HIP(hipMemsetAsync(B.acc, 0, sizeof(int64_t) * SPREAD * SPREAD_I64, st));
    if (m) {
        k_bip_volume<<<grid_for(m, BLOCK, REDUCE_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.nwgt, m, B.acc);
        HGP_LAUNCH_CHECK();
    }
    k_total<<<1, WAVE, 0, st>>>(B.acc, B.tot);
    HGP_LAUNCH_CHECK();
    int64_t half = 0;
    HGP_CHECK_HIP(hipMemcpyAsync(&half, B.tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    stream_sync(st);
    if (2 * half >= ((int64_t)1 << 31)) { A.release(mk); return HGP_E_INVALID; }
    const int64_t m2 = 2 * half;
    // level 0: G_x
    LvGraph *g = &B.G[0];
    if (m) {
        k_bip_nets<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, h.nwgt, n, m, p, g->pin_off,
                                                                     g->pins, g->inc_off, g->inc, g->vwgt, g->nwgt);
        HGP_LAUNCH_CHECK();
    } else {
        fill<uint32_t>(g->pin_off, 1, 0u, st);
        fill<uint32_t>(g->inc_off + n, 1, 0u, st);
    }
    k_bip_vertices<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, h.inc, h.pin_off, h.pins, h.nwgt, n,
                                                                     g->inc_off, g->inc, g->vwgt);
    HGP_LAUNCH_CHECK();
    k_iota<uint32_t><<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.node, n);
    HGP_LAUNCH_CHECK();
    hgp_hg cur{N, p, 2 * p, g->pin_off, g->pins, g->inc_off, g->inc, g->vwgt, g->nwgt};
    int which = 0;
    const uint64_t mseed = mix64(seed);
    uint32_t levels = 0;
    for (uint32_t level = 0; level < LV_LEVELS && m2 > 0; ++level) {
        const uint32_t Nc = cur.n;
        k_lv_init<<<grid_for(Nc, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(cur.vwgt, Nc, B.comm, B.cvol);
        HGP_LAUNCH_CHECK();
        HGP_CHECK_HIP(hipMemsetAsync(B.acc, 0, sizeof(int64_t) * SPREAD * SPREAD_I64 * LV_ROUNDS, st));
        const int cb = bits_for(Nc ? Nc - 1 : 0);
        const uint64_t cmask = cb >= 64 ? ~0ull : ((1ull << cb) - 1);
        // sub-round temporaries
        A.release(tmk);
        const size_t items_cap = 2 * (size_t)p;
        uint64_t *keys = A.alloc<uint64_t>(items_cap), *keys_alt = A.alloc<uint64_t>(items_cap);
        uint32_t *vals = A.alloc<uint32_t>(items_cap), *vals_alt = A.alloc<uint32_t>(items_cap);
        uint64_t *d_tot = A.alloc<uint64_t>(4);
        int64_t level_moves = 0;
        for (uint32_t r = 0; r < LV_ROUNDS; ++r) {
            int64_t *racc = B.acc + (size_t)r * SPREAD * SPREAD_I64;
            for (uint32_t s = 0; s < LV_SUBROUNDS; ++s) {
                scan_apply<uint64_t>(A, Nc, SelPack{cur.inc_off, mseed, level, r, s}, SelStore{B.list, B.ioff}, d_tot,
                                     st);
                uint64_t tot = 0;
                HGP_CHECK_HIP(hipMemcpyAsync(&tot, d_tot, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
                stream_sync(st);
                const uint32_t count = (uint32_t)(tot >> 32), items = (uint32_t)tot;
                if (count == 0) continue;
                HGP_REQUIRE(items <= items_cap, HGP_E_WORKSPACE);
                // nodes of few edges decide at once; the others sort their
                // (node, community) keys first
                fill<uint32_t>(B.nmid, 1, 0u, st);
                k_lv_direct<<<grid_for(count, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
                    B.list, count, cur.inc_off, cur.inc, cur.pin_off, cur.pins, cur.nwgt, B.comm, B.cvol, cur.vwgt,
                    m2, B.dec, B.mid, B.nmid);
                HGP_LAUNCH_CHECK();
                k_lv_wave<<<grid_for(count, LVW_WAVES, 1024), BLOCK, 0, st>>>(B.list, B.mid, B.nmid, cur.inc_off,
                                                                           cur.inc, cur.pins, cur.nwgt, B.comm,
                                                                           B.cvol, cur.vwgt, m2, B.dec);
                HGP_LAUNCH_CHECK();
                if (items) {
                    fill<uint32_t>(B.ioff + count, 1, items, st);
                    uint64_t *kk = keys;
                    uint32_t *vv = vals;
                    k_lv_emit<<<grid_for(count, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
                        B.list, B.ioff, count, cur.inc_off, cur.inc, cur.pin_off, cur.pins, cur.nwgt, B.comm, cb, kk,
                        vv);
                    HGP_LAUNCH_CHECK();
                    radix_sort_pairs<uint64_t>(A, &kk, &vv, kk == keys ? keys_alt : keys,
                                               vv == vals ? vals_alt : vals, items, 0,
                                               bits_for(count - 1) + cb, st);
                    k_lv_decide<<<grid_for(count, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
                        B.list, B.ioff, count, kk, vv, B.comm, B.cvol, cur.vwgt, m2, cmask, B.dec);
                    HGP_LAUNCH_CHECK();
                }
                k_lv_apply<<<grid_for(count, BLOCK, REDUCE_BLOCKS), BLOCK, 0, st>>>(B.list, B.dec, count, cur.vwgt,
                                                                                 B.comm, B.cvol, racc);
                HGP_LAUNCH_CHECK();
            }
            k_total<<<1, WAVE, 0, st>>>(racc, B.tot + r);
            HGP_LAUNCH_CHECK();
            int64_t mv = 0;
            HGP_CHECK_HIP(hipMemcpyAsync(&mv, B.tot + r, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            stream_sync(st);
            level_moves += mv;
            if (mv == 0) break;  // a round without moves ends the level
        }
        A.release(tmk);
        if (level_moves == 0) break;
        // contract every community into its smallest node
        fill<uint32_t>(B.minid, Nc, NONE, st);
        k_lv_minid<<<grid_for(Nc, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.comm, Nc, B.minid);
        HGP_LAUNCH_CHECK();
        k_lv_rep<<<grid_for(Nc, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.comm, B.minid, Nc, B.rep);
        HGP_LAUNCH_CHECK();
        LvGraph *nx = &B.G[1 - which];
        hgp_hg_out out;
        out.cap_n = N; out.cap_m = p; out.cap_p = 2 * p;
        out.pin_off = nx->pin_off; out.pins = nx->pins; out.inc_off = nx->inc_off; out.inc = nx->inc;
        out.vwgt = nx->vwgt; out.nwgt = nx->nwgt; out.dims = nullptr;
        uint32_t dims[3];
        contract(cur, B.rep, B.cid, out, dims, A, st);
        k_lv_map<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.cid, n, B.node);
        HGP_LAUNCH_CHECK();
        ++levels;
        const bool shrunk = dims[0] < Nc;
        cur = hgp_hg{dims[0], dims[1], dims[2], nx->pin_off, nx->pins, nx->inc_off, nx->inc, nx->vwgt, nx->nwgt};
        which = 1 - which;
        if (!shrunk) break;
    }
    HGP_CHECK_HIP(hipMemcpyAsync(comm_out, B.node, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
    stream_sync(st);
    if (levels_out) *levels_out = levels;
    A.release(mk);
    return HGP_OK;
}

}  // namespace hgp
