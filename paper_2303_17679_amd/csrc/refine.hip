// Deterministic synchronous label propagation (paper Sec. 11) on the
// connectivity objective (Sec. 2) with the connectivity gain of Sec. 6.
//
// Partition state per net (paper Sec. 6.1 keeps pin counts Phi(e,b) and the
// connectivity set Lambda(e) as a k-bit bitset).  Here every net stores two
// k-bit bitsets: Lambda(e) = {b : Phi(e,b) > 0} and Lambda1(e) = {b :
// Phi(e,b) = 1}.  These are exactly what the gain needs:
//   b(u)     = w({e in I(u) : Pi[u] in Lambda1(e)})
//   aff(u,t) = w({e in I(u) : t in Lambda(e)})
//   g_u(t)   = b(u) - (w(I(u)) - aff(u,t)).
// After a sub-round's moves are applied, the two bitsets of every net
// touching a moved node are recomputed from its pins (net-parallel, no
// atomics on counts), and the objective changes by
// sum over those nets of w(e) * (max(lambda'-1,0) - max(lambda-1,0)).
//
// Selection per block pair: proposals are sorted by (s, t, gain desc, u asc)
// with the stable radix sort; within a pair the paper's two-pointer walk is a
// merge of the two exclusive weight-prefix sequences (A first on ties), so
// the state after each step is found by one binary search in the other
// sequence and every element tests its own state in parallel; the last
// feasible state is an atomicMax over (step, i).
#include "prims.h"
#include "kernels.h"
#include "timing.h"

namespace hgp {

template <int KW>
struct Bits {
    uint64_t w[KW];
};

// Connectivity record of one net: Lambda (blocks holding a pin of the net)
// and Lambda1 (blocks holding exactly one pin) as k-bit sets, and the net
// weight.  A gain or an update that touches a net reads one record: 32 bytes
// for k <= 64, half of a 64-byte HBM sector, where three separate arrays
// would cost three sectors.
template <int KW>
struct alignas(16) NetRec {
    uint64_t lam[KW];
    uint64_t lam1[KW];
    int64_t w;
};
static_assert(sizeof(NetRec<1>) == 32 && sizeof(NetRec<2>) == 48 && sizeof(NetRec<4>) == 80, "record size");
inline size_t netrec_bytes(int KW) { return 16u * (size_t)(KW + 1); }

// Degree classes of LP candidates: lanes per node 1 (<= 8 nets), 8 (<= 64),
// a wave (<= HUB_DEG), a 1024-thread workgroup (more).
constexpr int NDEG = 4;
constexpr uint32_t HUB_DEG = 2048;
__host__ __device__ inline int deg_class(uint32_t d) { return d <= 8 ? 0 : (d <= 64 ? 1 : (d <= HUB_DEG ? 2 : 3)); }

// ---------------------------------------------------------------------------
// Connectivity bitsets of nets
// ---------------------------------------------------------------------------
template <int KW>
__device__ inline void net_bits(const uint32_t *pins, uint32_t b, uint32_t len, const uint32_t *part, uint64_t *once,
                                uint64_t *twice) {
#pragma unroll
    for (int q = 0; q < KW; ++q) { once[q] = 0; twice[q] = 0; }
    // eight pins at a time: all pin loads, then all block loads, then the fold
    for (uint32_t j0 = 0; j0 < len; j0 += 8) {
        uint32_t blk[8];
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) blk[c] = j0 + c < len ? pins[b + j0 + c] : NONE;
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) blk[c] = blk[c] != NONE ? part[blk[c]] : NONE;
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (blk[c] == NONE) continue;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint64_t bit = ((uint32_t)q == (blk[c] >> 6)) ? (1ull << (blk[c] & 63)) : 0ull;
                twice[q] |= once[q] & bit;
                once[q] |= bit;
            }
        }
    }
}

__device__ inline int64_t lam_cost(int lam) { return lam > 1 ? (int64_t)(lam - 1) : 0; }

template <int KW>
__device__ inline int popc_bits(const uint64_t *x) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < KW; ++q) c += __popcll(x[q]);
    return c;
}

// Control words of an LP level.  Every kernel of sub-round `stamp` (stamps
// 1 + r * S + s are consecutive over the level's rounds) does nothing once
// an earlier sub-round was handed to the device-wide path (abort holds its
// stamp) or when the previous round moved no node (prev -> its moves flag),
// so whole rounds are queued without a host round trip.
struct LpCtl {
    uint32_t *abort;
    const uint32_t *prev;  // nullptr in the first round
    uint32_t stamp;
};
__device__ inline bool lp_skip(const LpCtl &c) { return *c.abort != 0 || (c.prev && *c.prev == 0); }

// Thread per net for nets of at most 64 pins; longer nets go to a list.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_conn_small(const uint32_t *pin_off, const uint32_t *pins, uint32_t m,
                                                      const int32_t *nwgt, const uint32_t *part, NetRec<KW> *nr,
                                                      int64_t *f, uint32_t *longl, uint32_t *nlong,
                                                      uint64_t *cutbits) {
    __shared__ int64_t red[BLOCK / WAVE];
    int64_t acc = 0;
    for (uint32_t e0 = blockIdx.x * blockDim.x; e0 < m; e0 += gridDim.x * blockDim.x) {
        uint32_t e = e0 + threadIdx.x;
        bool act = e < m;
        uint32_t b = act ? pin_off[e] : 0, len = act ? pin_off[e + 1] - b : 0;
        bool lng = act && len > 64;
        uint32_t pos = warp_agg_append(nlong, lng);
        if (lng) longl[pos] = e;
        bool cut = false;
        if (act && !lng) {
            uint64_t once[KW], twice[KW];
            net_bits<KW>(pins, b, len, part, once, twice);
            NetRec<KW> R;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                R.lam[q] = once[q];
                R.lam1[q] = once[q] & ~twice[q];
            }
            R.w = nwgt[e];
            nr[e] = R;
            const int lam = popc_bits<KW>(once);
            acc += lam_cost(lam) * R.w;
            cut = lam > 1;
        }
        // one bit per net: cut or not (long nets are added by k_conn_long)
        const uint64_t word = __ballot(cut);
        const uint32_t ebase = e0 + (threadIdx.x & ~(WAVE - 1));
        if (__lane_id() == 0 && ebase < m) cutbits[ebase / WAVE] = word;
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
        if (t) spread_add_i64(f, t);
    }
}

// Wave per long net.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_conn_long(const uint32_t *pin_off, const uint32_t *pins,
                                                     const uint32_t *list, const uint32_t *count_dev,
                                                     const int32_t *nwgt, const uint32_t *part, NetRec<KW> *nr,
                                                     int64_t *f, bool delta, uint32_t *bcnt, LpCtl ctl,
                                                     uint32_t *cutbits = nullptr) {
    if (ctl.abort && lp_skip(ctl)) return;  // (no control words when building the records)
    const uint32_t count = *count_dev;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    for (uint32_t idx = wid; idx < count; idx += nw) {
        uint32_t e = list[idx];
        uint32_t b = pin_off[e], len = pin_off[e + 1] - b;
        uint64_t once[KW], twice[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) { once[q] = 0; twice[q] = 0; }
        for (uint32_t j = __lane_id(); j < len; j += WAVE) {
            uint32_t blk = part[pins[b + j]];
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                uint64_t bit = ((uint32_t)q == (blk >> 6)) ? (1ull << (blk & 63)) : 0ull;
                twice[q] |= once[q] & bit;
                once[q] |= bit;
            }
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                uint64_t oo = __shfl_xor(once[q], o, 64);
                uint64_t ot = __shfl_xor(twice[q], o, 64);
                twice[q] = twice[q] | ot | (once[q] & oo);
                once[q] |= oo;
            }
        }
        const int lnew = popc_bits<KW>(once);
        const int lold = delta ? popc_bits<KW>(nr[e].lam) : 0;  // read before lane 0 rewrites
        wave_sync();
        if (__lane_id() == 0) {
            int64_t d = lam_cost(lnew) - (delta ? lam_cost(lold) : 0);
            NetRec<KW> R;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                R.lam[q] = once[q];
                R.lam1[q] = once[q] & ~twice[q];
            }
            R.w = nwgt[e];
            nr[e] = R;
            if (d) spread_add_i64(f, d * R.w);
            if (cutbits && lnew > 1) atomicOr(&cutbits[e >> 5], 1u << (e & 31));
        }
        if (delta && bcnt && (lnew > 1) != (lold > 1)) {
            const uint32_t dl = lnew > 1 ? 1u : 0xFFFFFFFFu;
            for (uint32_t j = __lane_id(); j < len; j += WAVE) atomicAdd(&bcnt[pins[b + j]], dl);
        }
    }
}

// Largest net size of the level (one atomic per workgroup).
__global__ __launch_bounds__(BLOCK) void k_max_net(const uint32_t *pin_off, uint32_t m, uint32_t *out) {
    uint32_t mx = 0;
    for (uint32_t e = blockIdx.x * BLOCK + threadIdx.x; e < m; e += gridDim.x * BLOCK) {
        const uint32_t sz = pin_off[e + 1] - pin_off[e];
        mx = sz > mx ? sz : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(mx, o, WAVE);
        mx = y > mx ? y : mx;
    }
    __shared__ uint32_t red[BLOCK / WAVE];
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BLOCK / WAVE; ++q) mx = red[q] > mx ? red[q] : mx;
        if (mx) atomicMax(out, mx);
    }
}

// On a graph level every net has exactly two pins, so pin_off[e] = 2e and
// the kernels below read a net's endpoints at pins[2e] and pins[2e + 1]
// without loading the offsets.
// Adjacency array of a graph level: for the j-th incident net e of u,
// adj[j] = the other pin of e and adjw[j] = w(e).  A thread per vertex of up
// to 32 nets (eight incidence loads, then eight net loads at a time), the
// whole wave for up to ADJ_HEAVY nets; heavier vertices are listed for
// k_graph_adj_heavy.
constexpr uint32_t ADJ_HEAVY = 4096;
__global__ __launch_bounds__(BLOCK) void k_graph_adj(const uint32_t *inc_off, const uint32_t *inc,
                                                     const uint32_t *pin_off, const uint32_t *pins,
                                                     const int32_t *nwgt, uint32_t n, uint32_t *adj, int32_t *adjw,
                                                     uint32_t *heavy, uint32_t *nheavy) {
    for (uint32_t u0 = blockIdx.x * BLOCK; u0 < n; u0 += gridDim.x * BLOCK) {
        const uint32_t u = u0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (u < n) { j0 = inc_off[u]; j1 = inc_off[u + 1]; }
        const bool wide = j1 - j0 > 32;
        if (!wide)
            for (uint32_t j = j0; j < j1; j += 8) {
                uint32_t e[8];
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) e[q] = j + q < j1 ? inc[j + q] : NONE;
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) {
                    if (e[q] == NONE) continue;
                    const uint32_t x = pins[2 * (size_t)e[q]], y = pins[2 * (size_t)e[q] + 1];
                    adj[j + q] = x == u ? y : x;
                    adjw[j + q] = nwgt[e[q]];
                }
            }
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t hu = __shfl(u, h, WAVE), hj0 = __shfl(j0, h, WAVE), hj1 = __shfl(j1, h, WAVE);
            if (hj1 - hj0 > ADJ_HEAVY) {
                if ((int)__lane_id() == h) heavy[atomicAdd(nheavy, 1u)] = hu;
                continue;
            }
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) {
                const uint32_t e = inc[j], x = pins[2 * (size_t)e], y = pins[2 * (size_t)e + 1];
                adj[j] = x == hu ? y : x;
                adjw[j] = nwgt[e];
            }
        }
    }
}

// Listed heavy vertices, cut into chunks of ADJ_CHUNK incidence entries so
// that the grid is balanced whatever the degrees: cbase[i] (one workgroup)
// is the first chunk of listed vertex i, cbase[cnt] the number of chunks.
constexpr uint32_t ADJ_CHUNK = 4096;
constexpr int HEAVY_SCAN = 1024;
__global__ __launch_bounds__(HEAVY_SCAN) void k_heavy_chunks(const uint32_t *inc_off, const uint32_t *heavy,
                                                             const uint32_t *nheavy, uint32_t *cbase,
                                                             uint32_t chunk = ADJ_CHUNK) {
    __shared__ uint32_t red[HEAVY_SCAN / WAVE];
    const uint32_t cnt = *nheavy;
    uint32_t carry = 0;
    for (uint32_t i0 = 0; i0 < cnt; i0 += HEAVY_SCAN) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t c = 0;
        if (i < cnt) {
            const uint32_t u = heavy[i];
            c = (inc_off[u + 1] - inc_off[u] + chunk - 1) / chunk;
        }
        uint32_t tot;
        const uint32_t incl = block_incl_scan_n<uint32_t, HEAVY_SCAN>(c, red, &tot);
        if (i < cnt) cbase[i] = carry + incl - c;
        carry += tot;
    }
    if (threadIdx.x == 0) cbase[cnt] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_graph_adj_heavy(const uint32_t *inc_off, const uint32_t *inc,
                                                           const uint32_t *pin_off, const uint32_t *pins,
                                                           const int32_t *nwgt, const uint32_t *heavy,
                                                           const uint32_t *nheavy, const uint32_t *cbase,
                                                           uint32_t *adj, int32_t *adjw) {
    const uint32_t cnt = *nheavy, total = cbase[cnt];
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
        uint32_t lo = 0, hi = cnt;  // the listed vertex whose chunks hold g: last i with cbase[i] <= g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (cbase[mid] <= g) lo = mid; else hi = mid;
        }
        const uint32_t u = heavy[lo], j1 = inc_off[u + 1];
        const uint32_t jb = inc_off[u] + (g - cbase[lo]) * ADJ_CHUNK, je = jb + ADJ_CHUNK < j1 ? jb + ADJ_CHUNK : j1;
        for (uint32_t j = jb + threadIdx.x; j < je; j += BLOCK) {
            const uint32_t e = inc[j], x = pins[2 * (size_t)e], y = pins[2 * (size_t)e + 1];
            adj[j] = x == u ? y : x;
            adjw[j] = nwgt[e];
        }
    }
}

// Objective (edge cut) and cut bits of a graph level, a thread per edge.
__global__ __launch_bounds__(BLOCK) void k_conn_graph(const uint32_t *pin_off, const uint32_t *pins, uint32_t m,
                                                      const int32_t *nwgt, const uint32_t *part, int64_t *f,
                                                      uint64_t *cutbits) {
    __shared__ int64_t red[BLOCK / WAVE];
    int64_t acc = 0;
    for (uint32_t e0 = blockIdx.x * blockDim.x; e0 < m; e0 += gridDim.x * blockDim.x) {
        const uint32_t e = e0 + threadIdx.x;
        bool cut = false;
        if (e < m) {
            cut = part[pins[2 * (size_t)e]] != part[pins[2 * (size_t)e + 1]];
            if (cut) acc += nwgt[e];
        }
        const uint64_t word = __ballot(cut);
        const uint32_t ebase = e0 + (threadIdx.x & ~(WAVE - 1));
        if (__lane_id() == 0 && ebase < m) cutbits[ebase / WAVE] = word;
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
        if (t) spread_add_i64(f, t);
    }
}

__global__ __launch_bounds__(BLOCK) void k_block_weights(const uint32_t *part, const int32_t *vwgt, uint32_t n,
                                                         uint32_t k, int64_t *bw) {
    __shared__ int64_t h[256];
    for (uint32_t b = threadIdx.x; b < k; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        atomicAdd((unsigned long long *)&h[part[v]], (unsigned long long)(int64_t)vwgt[v]);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < k; b += blockDim.x)
        if (h[b]) atomic_add_i64(&bw[b], h[b]);
}

// ---------------------------------------------------------------------------
// Gains
// ---------------------------------------------------------------------------
template <int KW>
struct GainArgs {
    const uint32_t *inc_off, *inc;
    const int32_t *vwgt;
    const NetRec<KW> *nr;
    const uint32_t *part;
    const int64_t *bw;
    const uint32_t *bcnt;  // incident nets with lambda > 1 (boundary iff > 0)
    const int64_t *lmax;  // [k] weight limit of every block
    uint64_t mseed;
    uint32_t level, round, sub, S, n;
    uint32_t *prop_t, *prop_g;
    // proposals: NSLOT lists, list j (at plist + j * slot_cap, its length
    // in pcnt[j * SPREAD_U32]) holds the proposers of the vertex chunks
    // c = j (mod NSLOT), chunks of `ch` consecutive vertices
    uint32_t *plist, *pcnt;
    uint32_t ch, slot_cap;
    uint32_t *pw;  // [k*k] total weight proposed per ordered block pair
    uint32_t *pc;  // [k*k] number of proposals per ordered block pair
    uint32_t k;
    LpCtl ctl;
    // Graph levels (every net has two pins): adj[j] is the other endpoint of
    // the j-th incident net of its vertex and adjw[j] that net's weight, so a
    // gain reads the neighbour's block instead of a net record.  nullptr on
    // hypergraph levels.
    const uint32_t *adj = nullptr;
    const int32_t *adjw = nullptr;
};

// What a gain needs of incident net j of a vertex in block s: its weight,
// its Lambda words and the Lambda1 word that holds bit s (a memory read at a
// computed offset, never a local copy of the record: a dynamically indexed
// local array goes to scratch memory).  On a graph level (GR, a template
// parameter, so that neither kind of level pays for the other's loads) the
// net is an edge to a neighbour in block b: Lambda = {s, b}, and Lambda1 =
// Lambda when b differs from s, else empty.
template <int KW, bool GR>
__device__ inline void net_fields(const GainArgs<KW> &a, uint32_t j, uint32_t s, int64_t &w, uint64_t (&lam)[KW],
                                  uint64_t &one) {
    if constexpr (GR) {
        const uint32_t b = a.part[a.adj[j]];
        w = a.adjw[j];
        one = 0;
#pragma unroll
        for (int q = 0; q < KW; ++q) {
            lam[q] = (((uint32_t)q == (s >> 6)) ? (1ull << (s & 63)) : 0ull) |
                     (((uint32_t)q == (b >> 6)) ? (1ull << (b & 63)) : 0ull);
            if ((uint32_t)q == (s >> 6) && b != s) one = lam[q];
        }
    } else {
        const NetRec<KW> &R = a.nr[a.inc[j]];
        w = R.w;
#pragma unroll
        for (int q = 0; q < KW; ++q) lam[q] = R.lam[q];
        one = R.lam1[s >> 6];
    }
}

// Proposal lists: NSLOT lists by vertex chunk (see GainArgs).
constexpr uint32_t NSLOT = SPREAD;
static_assert(NSLOT == 64, "slot = XCD + 8 * (chunk mod 8)");

// List of vertex chunk c (of nchunks): the XCD whose share of the chunk
// range (xcd_slice over chunks) holds c, plus 8 (c mod 8).  Workgroup b
// reads list b mod NSLOT, and b mod 8 is its XCD, so a chunk's candidates
// are selected, rated, selected for moves and updated on one XCD: the net
// records that neighbouring chunks share stay in that XCD's L2.  A list
// holds at most chunk_slot_cap chunks.
__host__ __device__ inline uint32_t chunk_slot(uint32_t c, uint32_t nchunks) {
    uint32_t x = (uint32_t)((8ull * (c + 1) + nchunks - 1) / nchunks) - 1u;
    x = x < 7u ? x : 7u;
    return x + 8u * (c % 8u);
}
__host__ __device__ inline uint32_t chunk_slot_cap(uint32_t nchunks) { return ((nchunks + 7) / 8 + 7) / 8 + 1; }

// Called by every lane of the wave (uniformly); `has` is set by at most one
// lane per proposing vertex, and every proposing lane of the call belongs
// to list `slot`.
template <int KW>
__device__ inline void propose(const GainArgs<KW> &a, uint32_t u, uint32_t s, uint32_t t, uint32_t g, bool has,
                               uint32_t slot) {
    const uint32_t pos = warp_agg_append(&a.pcnt[slot * SPREAD_U32], has);
    if (has) {
        a.plist[(size_t)slot * a.slot_cap + pos] = u;
        a.prop_t[u] = t;
        a.prop_g[u] = g;
        atomicAdd(&a.pw[s * a.k + t], (uint32_t)a.vwgt[u]);
        atomicAdd(&a.pc[s * a.k + t], 1u);
    }
}

template <int G, class T>
__device__ inline T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Groups of G lanes per node (G = 1, 8 or 64 by degree class); the lanes of a
// group split the incident nets.  Best move: largest positive gain among the
// blocks of the union of Lambda(e), ties to the smaller block.  The list holds
// only candidates (boundary vertices of the sub-round).  For G < 64 a lane
// has at most 8 nets: their weight and Lambda words stay in registers for
// the per-target affinity sums, and all loads of a lane are issued before
// any is used.
template <int KW, int G, bool GR>
__device__ inline void gains_body(const GainArgs<KW> &a, const uint32_t *list, uint32_t count, uint32_t blk,
                                  uint32_t nblk, uint32_t slot, bool skip_inner = false) {
    constexpr int GPB = BLOCK / G;
    constexpr bool CACHE = G < 64;
    constexpr int NC = CACHE ? 8 : 1;
    const uint32_t g = threadIdx.x / G, l = threadIdx.x % G;
    const XcdSlice xs = xcd_slice(blk, nblk, count);
    for (uint32_t base = xs.lo + xs.wi * GPB; base < xs.hi; base += xs.nw * GPB) {
        const uint32_t idx = base + g;
        uint32_t u = 0, best_t = NONE, best_g = 0, s = 0;
        bool act = idx < xs.hi;
        if (act) u = list[idx];
        // (a vertex without a cut net has no other block in its nets: it
        // would propose nothing)
        if (act && skip_inner) act = a.bcnt[u] != 0;
        if (act) {  // uniform within the group
            const uint32_t j0 = a.inc_off[u], j1 = a.inc_off[u + 1];
            s = a.part[u];
            const int64_t cu = a.vwgt[u];
            int64_t bu = 0, wI = 0;
            uint64_t U[KW];
#pragma unroll
            for (int q = 0; q < KW; ++q) U[q] = 0;
            if constexpr (CACHE) {
                uint32_t ev[NC];
                int32_t wv[NC];
                uint64_t lv[NC][KW];
                // all incidence (or adjacency) loads, then all record (or
                // neighbour block) loads
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const uint32_t j = j0 + l + (uint32_t)c * G;
                    if constexpr (GR) {
                        ev[c] = j < j1 ? a.adj[j] : NONE;
                        wv[c] = j < j1 ? a.adjw[j] : 0;
                    } else {
                        ev[c] = j < j1 ? a.inc[j] : NONE;
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    uint64_t one = 0;
                    if constexpr (!GR) wv[c] = 0;
#pragma unroll
                    for (int q = 0; q < KW; ++q) lv[c][q] = 0;
                    if (ev[c] != NONE) {
                        if constexpr (GR) {
                            const uint32_t b = a.part[ev[c]];
#pragma unroll
                            for (int q = 0; q < KW; ++q) {
                                const uint64_t bits = (((uint32_t)q == (s >> 6)) ? (1ull << (s & 63)) : 0ull) |
                                                      (((uint32_t)q == (b >> 6)) ? (1ull << (b & 63)) : 0ull);
                                lv[c][q] = bits;
                                if ((uint32_t)q == (s >> 6)) one = b != s ? bits : 0ull;
                            }
                        } else {
                            const NetRec<KW> &R = a.nr[ev[c]];
                            wv[c] = (int32_t)R.w;
#pragma unroll
                            for (int q = 0; q < KW; ++q) lv[c][q] = R.lam[q];
                            one = R.lam1[s >> 6];
                        }
                    }
                    wI += wv[c];
                    if ((one >> (s & 63)) & 1ull) bu += wv[c];
#pragma unroll
                    for (int q = 0; q < KW; ++q) U[q] |= lv[c][q];
                }
                bu = group_sum<G>(bu);
                wI = group_sum<G>(wI);
#pragma unroll
                for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
                    for (int q = 0; q < KW; ++q) U[q] |= __shfl_xor(U[q], o, 64);
#pragma unroll
                for (int q = 0; q < KW; ++q)  // (a register array: no computed index)
                    if ((uint32_t)q == (s >> 6)) U[q] &= ~(1ull << (s & 63));
#pragma unroll
                for (int q = 0; q < KW; ++q) {
                    uint64_t x = U[q];
                    while (x) {
                        const int bit = __ffsll((long long)x) - 1;
                        x &= x - 1;
                        const uint32_t t = (uint32_t)(q * 64 + bit);
                        if (a.bw[t] + cu > a.lmax[t]) continue;
                        int64_t aff = 0;
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            if ((lv[c][q] >> bit) & 1ull) aff += wv[c];
                        aff = group_sum<G>(aff);
                        const int64_t gn = bu - (wI - aff);
                        if (gn > (int64_t)best_g) { best_g = (uint32_t)gn; best_t = t; }
                    }
                }
            } else {
                // one wave per node: the affinity of every block in one pass
                // over the incident nets (per-wave LDS histogram), so a node
                // of high degree costs sum of lambda(e), not degree x blocks
                static_assert(G == WAVE, "the histogram path is wave per node");
                __shared__ int64_t affs[BLOCK / WAVE][64 * KW];
                int64_t *aff = affs[g];
#pragma unroll
                for (int q = 0; q < KW; ++q) aff[q * 64 + l] = 0;
                wave_sync();
                for (uint32_t j = j0 + l; j < j1; j += G) {
                    int64_t w;
                    uint64_t lam[KW], one;
                    net_fields<KW, GR>(a, j, s, w, lam, one);
                    wI += w;
                    if ((one >> (s & 63)) & 1ull) bu += w;
#pragma unroll
                    for (int q = 0; q < KW; ++q) {
                        uint64_t x = lam[q];
                        U[q] |= x;
                        while (x) {
                            const int bit = __ffsll((long long)x) - 1;
                            x &= x - 1;
                            atomicAdd((unsigned long long *)&aff[q * 64 + bit], (unsigned long long)w);
                        }
                    }
                }
                bu = group_sum<G>(bu);
                wI = group_sum<G>(wI);
#pragma unroll
                for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
                    for (int q = 0; q < KW; ++q) U[q] |= __shfl_xor(U[q], o, 64);
#pragma unroll
                for (int q = 0; q < KW; ++q)  // (a register array: no computed index)
                    if ((uint32_t)q == (s >> 6)) U[q] &= ~(1ull << (s & 63));
                wave_sync();  // every histogram update is done
                // lane l judges blocks q * 64 + l (ascending per lane)
#pragma unroll
                for (int q = 0; q < KW; ++q) {
                    const uint32_t t = (uint32_t)(q * 64) + l;
                    if (!((U[q] >> l) & 1ull) || a.bw[t] + cu > a.lmax[t]) continue;
                    const int64_t gn = bu - (wI - aff[t]);
                    if (gn > (int64_t)best_g) { best_g = (uint32_t)gn; best_t = t; }
                }
                // largest gain, then smallest block
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const uint32_t og = __shfl_xor(best_g, o, 64), ot = __shfl_xor(best_t, o, 64);
                    if (og > best_g || (og == best_g && ot < best_t)) { best_g = og; best_t = ot; }
                }
                wave_sync();  // the histogram is read before the next node clears it
            }
        }
        propose(a, u, s, best_t, best_g, act && l == 0 && best_t != NONE, slot);
    }
}

// Candidates of LP sub-round (r, s): the boundary vertices (an incident net
// with lambda > 1 -- no other vertex can have a positive gain) whose
// sub-round hash selects s.  Each workgroup takes chunks of `ch` consecutive
// vertices (the chunks of one XCD are contiguous), gathers the chunk's
// candidates in LDS by degree class (1 lane per node up to 8 nets, 8 lanes up
// to 64, a wave up to HUB_DEG; larger nodes go to the hub list for
// k_gains_hub) and appends them to the class list of the chunk's slot
// c mod NSLOT (cl[class][slot], capacity slot_cap each, lengths in ccnt), one
// atomic per class and chunk.  Block 0 also clears the counters that only
// the later kernels of the sub-round use.
constexpr uint32_t GAIN_CH = 1024;  // largest chunk
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_gain_scan(GainArgs<KW> a, uint32_t ch, uint32_t nchunks, uint32_t *cl,
                                                     uint32_t *ccnt, uint32_t *hubl, uint32_t *nhub, uint32_t *scal) {
    __shared__ uint32_t lst[3][GAIN_CH];
    __shared__ uint32_t lcnt[3], lbase[3];
    if (lp_skip(a.ctl)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[2] = 0; scal[3] = 0;     // ntouched, nlong
        scal[13] = 0; scal[14] = 0;   // oversized-pair proposals, movers
        scal[24] = 0;                 // movers of more than HUB_DEG nets
    }
    const size_t cstride = (size_t)NSLOT * a.slot_cap;  // one class's lists
    const XcdSlice xs = xcd_slice(blockIdx.x, gridDim.x, nchunks);
    for (uint32_t c = xs.lo + xs.wi; c < xs.hi; c += xs.nw) {
        const uint32_t lo = c * ch, hi = lo + ch < a.n ? lo + ch : a.n;
        if (threadIdx.x < 3) lcnt[threadIdx.x] = 0;
        __syncthreads();
        // a thread's vertices lo + q * BLOCK: every load of a step is issued
        // before any is used (boundary counts, then the candidates' degrees)
        constexpr int PER = GAIN_CH / BLOCK;
        uint32_t bc[PER], d[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t v = lo + q * BLOCK + threadIdx.x;
            bc[q] = v < hi ? a.bcnt[v] : 0u;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t v = lo + q * BLOCK + threadIdx.x;
            if (bc[q] && tag_hash(a.mseed, 3, a.level, a.round, v) % a.S != a.sub) bc[q] = 0;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t v = lo + q * BLOCK + threadIdx.x;
            d[q] = bc[q] ? a.inc_off[v + 1] - a.inc_off[v] : 0u;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (!bc[q]) continue;
            const uint32_t v = lo + q * BLOCK + threadIdx.x;
            const int cls = deg_class(d[q]);
            if (cls == 3) hubl[atomicAdd(nhub, 1u)] = v;
            else lst[cls][atomicAdd(&lcnt[cls], 1u)] = v;
        }
        __syncthreads();
        const uint32_t slot = chunk_slot(c, nchunks);
        if (threadIdx.x < 3)
            lbase[threadIdx.x] =
                lcnt[threadIdx.x] ? atomicAdd(&ccnt[(threadIdx.x * NSLOT + slot) * SPREAD_U32], lcnt[threadIdx.x]) : 0u;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            uint32_t *dst = cl + t * cstride + (size_t)slot * a.slot_cap + lbase[t];
            for (uint32_t i = threadIdx.x; i < lcnt[t]; i += BLOCK) dst[i] = lst[t][i];
        }
        __syncthreads();  // the lists are rewritten by the next chunk
    }
}

// Gains of the listed candidates: workgroup b rates part of slot b mod
// NSLOT's class lists (the grid is a multiple of NSLOT), so every candidate
// of the sub-round is in flight at once, not a chunk's worth per workgroup.
// Resident workgroups per CU: six at one Lambda word (at most 80 registers);
// more words keep more per-lane registers (8 nets x KW words), so fewer
// workgroups rather than spills to scratch memory.
template <int KW>
constexpr int gains_occupancy() { return KW == 1 ? 6 : (KW == 2 ? 4 : 3); }

// poff == nullptr: the candidate lists of k_gain_scan (cl, ccnt).  Otherwise
// the lists of the level built by k_lp_pre: the vertices of class c and slot
// sl are cl[poff[c * NSLOT + sl] .. poff[c * NSLOT + sl + 1]), every vertex
// of the sub-round whether or not it has a cut net (those without are
// skipped), and block 0 clears the counters that k_gain_scan would.
template <int KW, bool GR>
__global__ __launch_bounds__(BLOCK, gains_occupancy<KW>()) void k_gains(GainArgs<KW> a, const uint32_t *cl,
                                                                        const uint32_t *ccnt, const uint32_t *poff,
                                                                        uint32_t *scal) {
    if (lp_skip(a.ctl)) return;
    const uint32_t sl = blockIdx.x % NSLOT, bj = blockIdx.x / NSLOT, nbj = gridDim.x / NSLOT;
    if (poff) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[2] = 0; scal[3] = 0;
            scal[13] = 0; scal[14] = 0;
            scal[24] = 0;
        }
        const uint32_t o0 = poff[sl], o1 = poff[NSLOT + sl], o2 = poff[2 * NSLOT + sl];
        gains_body<KW, 1, GR>(a, cl + o0, poff[sl + 1] - o0, bj, nbj, sl, true);
        gains_body<KW, 8, GR>(a, cl + o1, poff[NSLOT + sl + 1] - o1, bj, nbj, sl, true);
        gains_body<KW, 64, GR>(a, cl + o2, poff[2 * NSLOT + sl + 1] - o2, bj, nbj, sl, true);
        return;
    }
    const size_t cstride = (size_t)NSLOT * a.slot_cap;
    const size_t off = (size_t)sl * a.slot_cap;
    gains_body<KW, 1, GR>(a, cl + off, ccnt[(0 * NSLOT + sl) * SPREAD_U32], bj, nbj, sl);
    gains_body<KW, 8, GR>(a, cl + cstride + off, ccnt[(1 * NSLOT + sl) * SPREAD_U32], bj, nbj, sl);
    gains_body<KW, 64, GR>(a, cl + 2 * cstride + off, ccnt[(2 * NSLOT + sl) * SPREAD_U32], bj, nbj, sl);
}

// Candidate lists of every LP sub-round of a small level, built once per
// level instead of a selection launch per sub-round (on small levels the
// launches, not the bytes, bound a sub-round).  Key
// ((r * S + s) * 3 + c) * NSLOT + sl: round r, its sub-round s (the
// sub-round hash), degree class c, and the slot of the vertex's chunk (as
// k_gain_scan assigns it).  Every vertex with an incident net is listed once
// per round.  cur == nullptr: adds the count of every key to cnt; otherwise
// writes the vertices at the positions reserved from cur.  A workgroup takes
// one chunk at a time and BLOCK (vertex, round) pairs of it per step; one
// global atomic per key and step.
constexpr uint32_t LP_PRE_N = 1u << 17;  // levels of fewer vertices
constexpr uint32_t LP_PRE_RS = 64;       // rounds x sub-rounds at most
__global__ __launch_bounds__(BLOCK) void k_lp_pre(const uint32_t *inc_off, uint32_t n, uint64_t mseed,
                                                  uint32_t level, uint32_t R, uint32_t S, uint32_t ch,
                                                  uint32_t nchunks, uint32_t *cnt, uint32_t *cur,
                                                  uint32_t *lists) {
    __shared__ uint32_t lc[LP_PRE_RS * 3], lb[LP_PRE_RS * 3];
    const uint32_t nk = R * S * 3;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t lo = c * ch, len = (lo + ch < n ? lo + ch : n) - lo;
        const uint32_t slot = chunk_slot(c, nchunks);
        for (uint32_t q0 = 0; q0 < len * R; q0 += BLOCK) {
            for (uint32_t t = threadIdx.x; t < nk; t += BLOCK) lc[t] = 0;
            __syncthreads();
            const uint32_t q = q0 + threadIdx.x;
            uint32_t v = 0, key = NONE, rank = 0;
            if (q < len * R) {
                const uint32_t r = q / len;
                v = lo + q % len;
                const uint32_t d = inc_off[v + 1] - inc_off[v];
                if (d) {
                    const uint32_t sub = (uint32_t)(tag_hash(mseed, 3, level, r, v) % S);
                    key = (r * S + sub) * 3 + (uint32_t)deg_class(d);
                    rank = atomicAdd(&lc[key], 1u);
                }
            }
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < nk; t += BLOCK)
                if (lc[t]) {
                    if (cur) lb[t] = atomicAdd(&cur[t * NSLOT + slot], lc[t]);
                    else atomicAdd(&cnt[t * NSLOT + slot], lc[t]);
                }
            __syncthreads();
            if (cur && key != NONE) lists[lb[key] + rank] = v;
            __syncthreads();
        }
    }
}

// Exclusive prefix of the nk counts (one workgroup): off[i] and cur[i], and
// off[nk] = the total.
__global__ __launch_bounds__(BLOCK) void k_lp_pre_scan(const uint32_t *cnt, uint32_t nk, uint32_t *off,
                                                       uint32_t *cur) {
    __shared__ uint32_t wsum[BLOCK / WAVE];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nk; b += BLOCK) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < nk ? cnt[i] : 0u;
        uint32_t tot;
        const uint32_t incl = block_incl_scan<uint32_t>(v, wsum, &tot);
        if (i < nk) {
            off[i] = carry + incl - v;
            cur[i] = carry + incl - v;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) off[nk] = carry;
}

// Candidates of more than HUB_DEG nets: one 1024-thread workgroup each, the
// affinity of every block summed in a shared LDS histogram.
constexpr int HUB_THREADS = 1024;
template <int KW, bool GR>
__global__ __launch_bounds__(HUB_THREADS) void k_gains_hub(GainArgs<KW> a, const uint32_t *list,
                                                           const uint32_t *count_dev) {
    constexpr int NW = HUB_THREADS / WAVE;
    __shared__ int64_t aff[64 * KW];
    __shared__ unsigned long long Us[KW];
    __shared__ int64_t rbu[NW], rwi[NW];
    __shared__ uint32_t rg[NW], rt[NW];
    if (lp_skip(a.ctl)) return;
    const uint32_t cnt = *count_dev, tid = threadIdx.x, w = tid / WAVE;
    for (uint32_t idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        const uint32_t u = list[idx];
        const uint32_t j0 = a.inc_off[u], j1 = a.inc_off[u + 1];
        const uint32_t s = a.part[u];
        const int64_t cu = a.vwgt[u];
        for (uint32_t t = tid; t < 64 * KW; t += HUB_THREADS) aff[t] = 0;
        if (tid < KW) Us[tid] = 0;
        __syncthreads();
        int64_t bu = 0, wI = 0;
        uint64_t U[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) U[q] = 0;
        for (uint32_t j = j0 + tid; j < j1; j += HUB_THREADS) {
            int64_t wt;
            uint64_t lam[KW], one;
            net_fields<KW, GR>(a, j, s, wt, lam, one);
            wI += wt;
            if ((one >> (s & 63)) & 1ull) bu += wt;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                uint64_t x = lam[q];
                U[q] |= x;
                while (x) {
                    const int bit = __ffsll((long long)x) - 1;
                    x &= x - 1;
                    atomicAdd((unsigned long long *)&aff[q * 64 + bit], (unsigned long long)wt);
                }
            }
        }
        bu = wave_sum(bu);
        wI = wave_sum(wI);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int q = 0; q < KW; ++q) U[q] |= __shfl_xor(U[q], o, 64);
        if (__lane_id() == 0) {
            rbu[w] = bu;
            rwi[w] = wI;
#pragma unroll
            for (int q = 0; q < KW; ++q) atomicOr(&Us[q], (unsigned long long)U[q]);
        }
        __syncthreads();
        bu = 0;
        wI = 0;
        for (int q = 0; q < NW; ++q) { bu += rbu[q]; wI += rwi[q]; }
        uint32_t best_t = NONE, best_g = 0;
        if (tid < 64 * KW) {  // thread t judges block t
            const uint32_t t = tid;
            const bool inU = (Us[t >> 6] >> (t & 63)) & 1ull;
            if (inU && t != s && a.bw[t] + cu <= a.lmax[t]) {
                const int64_t gn = bu - (wI - aff[t]);
                if (gn > 0) { best_g = (uint32_t)gn; best_t = t; }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {  // largest gain, then smallest block
            const uint32_t og = __shfl_xor(best_g, o, 64), ot = __shfl_xor(best_t, o, 64);
            if (og > best_g || (og == best_g && ot < best_t)) { best_g = og; best_t = ot; }
        }
        if (__lane_id() == 0) { rg[w] = best_g; rt[w] = best_t; }
        __syncthreads();
        if (w == 0) {
            best_g = __lane_id() < NW ? rg[__lane_id()] : 0u;
            best_t = __lane_id() < NW ? rt[__lane_id()] : NONE;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t og = __shfl_xor(best_g, o, 64), ot = __shfl_xor(best_t, o, 64);
                if (og > best_g || (og == best_g && ot < best_t)) { best_g = og; best_t = ot; }
            }
            propose(a, u, s, best_t, best_g, __lane_id() == 0 && best_t != NONE,
                    chunk_slot(u / a.ch, (a.n + a.ch - 1) / a.ch));
        }
        __syncthreads();  // the histogram is read before the next node clears it
    }
}

// Hub gains summed by the whole grid: the incidence lists of the listed
// nodes are cut into chunks of HUB_GCH nets (cbase from k_heavy_chunks), a
// workgroup adds a chunk's block affinities, b(u), w(I(u)) and union of
// Lambda into the node's accumulators (integer atomics, so the sums do not
// depend on the order), and k_gains_hub_pick judges every node's blocks from
// them and clears them for the next sub-round.  Accumulator i: hacc[i *
// (64 KW + 2) + t] = affinity of block t, then b(u) and w(I(u)); hU[i * KW +
// q] = Lambda union words.
constexpr uint32_t HUB_GCH = 8192;
template <int KW, bool GR>
__global__ __launch_bounds__(HUB_THREADS) void k_gains_hub_part(GainArgs<KW> a, const uint32_t *list,
                                                                const uint32_t *count_dev, const uint32_t *cbase,
                                                                int64_t *hacc, unsigned long long *hU) {
    constexpr int NW = HUB_THREADS / WAVE;
    constexpr uint32_t ROW = 64 * KW + 2;
    __shared__ int64_t aff[64 * KW];
    __shared__ unsigned long long Us[KW];
    __shared__ int64_t rbu[NW], rwi[NW];
    if (lp_skip(a.ctl)) return;
    const uint32_t cnt = *count_dev, total = cbase[cnt], tid = threadIdx.x, w = tid / WAVE;
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {  // uniform per block
        uint32_t lo = 0, hi = cnt;  // the listed node whose chunks hold g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (cbase[mid] <= g) lo = mid; else hi = mid;
        }
        const uint32_t u = list[lo], j1 = a.inc_off[u + 1];
        const uint32_t jb = a.inc_off[u] + (g - cbase[lo]) * HUB_GCH, je = jb + HUB_GCH < j1 ? jb + HUB_GCH : j1;
        const uint32_t s = a.part[u];
        for (uint32_t t = tid; t < 64 * KW; t += HUB_THREADS) aff[t] = 0;
        if (tid < KW) Us[tid] = 0;
        __syncthreads();
        int64_t bu = 0, wI = 0;
        uint64_t U[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) U[q] = 0;
        for (uint32_t j = jb + tid; j < je; j += HUB_THREADS) {
            int64_t wt;
            uint64_t lam[KW], one;
            net_fields<KW, GR>(a, j, s, wt, lam, one);
            wI += wt;
            if ((one >> (s & 63)) & 1ull) bu += wt;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                uint64_t x = lam[q];
                U[q] |= x;
                while (x) {
                    const int bit = __ffsll((long long)x) - 1;
                    x &= x - 1;
                    atomicAdd((unsigned long long *)&aff[q * 64 + bit], (unsigned long long)wt);
                }
            }
        }
        bu = wave_sum(bu);
        wI = wave_sum(wI);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int q = 0; q < KW; ++q) U[q] |= __shfl_xor(U[q], o, 64);
        if (__lane_id() == 0) {
            rbu[w] = bu;
            rwi[w] = wI;
#pragma unroll
            for (int q = 0; q < KW; ++q) atomicOr(&Us[q], (unsigned long long)U[q]);
        }
        __syncthreads();
        int64_t *acc = hacc + (size_t)lo * ROW;
        for (uint32_t t = tid; t < 64 * KW; t += HUB_THREADS)
            if (aff[t]) atomic_add_i64(&acc[t], aff[t]);
        if (tid == 0) {
            int64_t tb = 0, tw = 0;
            for (int q = 0; q < NW; ++q) { tb += rbu[q]; tw += rwi[q]; }
            if (tb) atomic_add_i64(&acc[64 * KW], tb);
            if (tw) atomic_add_i64(&acc[64 * KW + 1], tw);
        }
        if (tid < KW && Us[tid]) atomicOr(&hU[(size_t)lo * KW + tid], Us[tid]);
        __syncthreads();  // the LDS sums are read before the next chunk clears them
    }
}

template <int KW>
__global__ __launch_bounds__(BLOCK) void k_gains_hub_pick(GainArgs<KW> a, const uint32_t *list,
                                                          const uint32_t *count_dev, int64_t *hacc,
                                                          unsigned long long *hU) {
    constexpr uint32_t ROW = 64 * KW + 2;
    static_assert(64 * KW <= BLOCK, "a thread per block");
    __shared__ uint32_t rg[BLOCK / WAVE], rt[BLOCK / WAVE];
    if (lp_skip(a.ctl)) return;
    const uint32_t cnt = *count_dev, tid = threadIdx.x, w = tid / WAVE;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {  // uniform per block
        const uint32_t u = list[i], s = a.part[u];
        const int64_t cu = a.vwgt[u];
        int64_t *acc = hacc + (size_t)i * ROW;
        const int64_t bu = acc[64 * KW], wI = acc[64 * KW + 1];
        uint32_t best_t = NONE, best_g = 0;
        if (tid < 64 * KW) {  // thread t judges block t
            const uint32_t t = tid;
            const bool inU = (hU[(size_t)i * KW + (t >> 6)] >> (t & 63)) & 1ull;
            if (inU && t != s && a.bw[t] + cu <= a.lmax[t]) {
                const int64_t gn = bu - (wI - acc[t]);
                if (gn > 0) { best_g = (uint32_t)gn; best_t = t; }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {  // largest gain, then smallest block
            const uint32_t og = __shfl_xor(best_g, o, 64), ot = __shfl_xor(best_t, o, 64);
            if (og > best_g || (og == best_g && ot < best_t)) { best_g = og; best_t = ot; }
        }
        if (__lane_id() == 0) { rg[w] = best_g; rt[w] = best_t; }
        __syncthreads();
        // clear the accumulators for the next sub-round (every read is done)
        for (uint32_t t = tid; t < ROW; t += BLOCK) acc[t] = 0;
        if (tid < KW) hU[(size_t)i * KW + tid] = 0;
        if (w == 0) {
            best_g = __lane_id() < BLOCK / WAVE ? rg[__lane_id()] : 0u;
            best_t = __lane_id() < BLOCK / WAVE ? rt[__lane_id()] : NONE;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t og = __shfl_xor(best_g, o, 64), ot = __shfl_xor(best_t, o, 64);
                if (og > best_g || (og == best_g && ot < best_t)) { best_g = og; best_t = ot; }
            }
            propose(a, u, s, best_t, best_g, __lane_id() == 0 && best_t != NONE,
                    chunk_slot(u / a.ch, (a.n + a.ch - 1) / a.ch));
        }
        __syncthreads();
    }
}

// The same count with a wave per node, for levels whose average degree is
// high (coarse levels).
// Nodes of more than BCNT_HUGE nets are counted by a workgroup each.
constexpr uint32_t BCNT_HUGE = 8192;
constexpr int BCNT_HUGE_THREADS = 1024;
__global__ __launch_bounds__(BCNT_HUGE_THREADS) void k_init_bcnt_huge(const uint32_t *inc_off, const uint32_t *inc,
                                                                      const uint32_t *cut, const uint32_t *huge,
                                                                      const uint32_t *nhuge, uint32_t *bcnt) {
    __shared__ uint32_t red[BCNT_HUGE_THREADS / WAVE];
    const uint32_t cnt = *nhuge;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {  // uniform per block
        const uint32_t u = huge[i], j1 = inc_off[u + 1];
        uint32_t t = 0;
        for (uint32_t j = inc_off[u] + threadIdx.x; j < j1; j += BCNT_HUGE_THREADS) {
            const uint32_t e = inc[j];
            t += (cut[e >> 5] >> (e & 31)) & 1u;
        }
        t = wave_sum(t);
        if (__lane_id() == 0) red[threadIdx.x / WAVE] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < BCNT_HUGE_THREADS / WAVE; ++q) t += red[q];
            bcnt[u] = t;
        }
        __syncthreads();
    }
}

template <int KW>
__global__ __launch_bounds__(BLOCK) void k_init_bcnt_wave(const uint32_t *inc_off, const uint32_t *inc, uint32_t n,
                                                          const uint32_t *cut, uint32_t *bcnt, uint32_t *huge,
                                                          uint32_t *nhuge) {
    const uint32_t wid = (blockIdx.x * BLOCK + threadIdx.x) / WAVE, nw = gridDim.x * BLOCK / WAVE;
    for (uint32_t u = wid; u < n; u += nw) {
        const uint32_t j0 = inc_off[u], j1 = inc_off[u + 1];
        if (j1 - j0 > BCNT_HUGE) {  // uniform per wave: a workgroup counts it (k_init_bcnt_huge)
            if (__lane_id() == 0) huge[atomicAdd(nhuge, 1u)] = u;
            continue;
        }
        uint32_t t = 0;
        for (uint32_t j = j0 + __lane_id(); j < j1; j += WAVE) {
            const uint32_t e = inc[j];
            t += (cut[e >> 5] >> (e & 31)) & 1u;
        }
        t = wave_sum(t);
        if (__lane_id() == 0) bcnt[u] = t;
    }
}

// Boundary count of every node from scratch (once per level), from the bit
// per net that the connectivity kernels leave (the bitmap is small enough to
// stay in L2); a node of more than 32 nets is counted by its whole wave.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_init_bcnt(const uint32_t *inc_off, const uint32_t *inc, uint32_t n,
                                                     const uint32_t *cut, uint32_t *bcnt) {
    for (uint32_t u0 = blockIdx.x * BLOCK; u0 < n; u0 += gridDim.x * BLOCK) {
        const uint32_t u = u0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (u < n) { j0 = inc_off[u]; j1 = inc_off[u + 1]; }
        const bool heavy = j1 - j0 > 32;
        uint32_t c = 0;
        if (!heavy)  // eight nets at a time: all incidence loads, then all record loads
            for (uint32_t j = j0; j < j1; j += 8) {
                uint32_t e[8];
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) e[q] = j + q < j1 ? inc[j + q] : NONE;
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) c += e[q] != NONE ? (cut[e[q] >> 5] >> (e[q] & 31)) & 1u : 0u;
            }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int h = __ffsll((long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t hj0 = __shfl(j0, h, 64), hj1 = __shfl(j1, h, 64);
            uint32_t t = 0;
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) {
                const uint32_t e = inc[j];
                t += (cut[e >> 5] >> (e & 31)) & 1u;
            }
            t = wave_sum(t);
            if ((int)__lane_id() == h) c = t;
        }
        if (u < n) bcnt[u] = c;
    }
}

// Measurement only: compulsory bytes of one gains launch: the boundary
// count of every vertex; for every boundary vertex the sub-round selects, its
// incidence offsets (and a hub-list entry for the nodes left to k_gains_hub);
// for every candidate it rates, its block, weight and incidence list; for
// every distinct incident net of those its weight, Lambda words and the one
// Lambda1 word the gain reads, counted once.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_account_gains(GainArgs<KW> a, uint32_t *nmark, uint32_t stamp,
                                                         unsigned long long *acc) {
    __shared__ unsigned long long red[BLOCK / WAVE];
    if (lp_skip(a.ctl)) return;  // the sub-round does nothing
    unsigned long long bytes = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        // the candidates of k_gains (k_gain_scan's boundary counts and the
        // hub candidates are not its bytes)
        if (a.bcnt[v] == 0 || tag_hash(a.mseed, 3, a.level, a.round, v) % a.S != a.sub) continue;
        const uint32_t j0 = a.inc_off[v], j1 = a.inc_off[v + 1];
        if (deg_class(j1 - j0) == 3) continue;
        bytes += 4 + 8 + 4 + 4 + 4ull * (j1 - j0);  // list entry, offsets, block, weight, incidence list
        for (uint32_t j = j0; j < j1; ++j)
            if (atomicExch(&nmark[a.inc[j]], stamp) != stamp) bytes += 4 + 8ull * KW + 8;
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

// Vertices per degree class (deg_class; degree-0 vertices are in none):
// sizes the candidate lists of the level.
__global__ __launch_bounds__(BLOCK) void k_deg_classify(const uint32_t *inc_off, uint32_t n, uint32_t *counts) {
    __shared__ uint32_t lcnt[NDEG];
    if (threadIdx.x < NDEG) lcnt[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t u = blockIdx.x * BLOCK + threadIdx.x; u < n; u += gridDim.x * BLOCK) {
        const uint32_t d = inc_off[u + 1] - inc_off[u];
        if (d > 0) atomicAdd(&lcnt[deg_class(d)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NDEG && lcnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], lcnt[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Pair sort keys, segment bounds, selection, apply
// ---------------------------------------------------------------------------
struct KeyLayout {
    int sh_s, sh_t, sh_g, sh_u;  // bit positions
    uint32_t kmask;
    uint32_t G;  // gmax: stored as G - g (descending gain)
    bool with_u;
};

__global__ void k_lp_keys(const uint32_t *plist, uint32_t np, const uint32_t *part, const uint32_t *prop_t,
                          const uint32_t *prop_g, KeyLayout L, uint64_t *keys, uint32_t *vals, bool from_vals) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        uint32_t u = from_vals ? vals[i] : plist[i];
        uint64_t key = ((uint64_t)part[u] << L.sh_s) | ((uint64_t)prop_t[u] << L.sh_t) |
                       ((uint64_t)(L.G - prop_g[u]) << L.sh_g);
        if (L.with_u) key |= (uint64_t)u << L.sh_u;
        keys[i] = key;
        vals[i] = u;
    }
}

__global__ void k_u_only_keys(const uint32_t *plist, uint32_t np, uint64_t *keys, uint32_t *vals) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        keys[i] = plist[i];
        vals[i] = plist[i];
    }
}

struct SortedWeight {
    const uint32_t *vals;
    const int32_t *vwgt;
    __device__ uint64_t operator()(size_t i) const { return (uint64_t)(uint32_t)vwgt[vals[i]]; }
};
struct StoreIncl {
    uint64_t *out;
    __device__ void operator()(size_t i, uint64_t excl, uint64_t v) const { out[i] = excl + v; }
};

__device__ inline uint32_t key_pair(uint64_t key, const KeyLayout &L, uint32_t k) {
    uint32_t s = (uint32_t)(key >> L.sh_s) & L.kmask;
    uint32_t t = (uint32_t)(key >> L.sh_t) & L.kmask;
    return s * k + t;
}

__global__ void k_pair_bounds(const uint64_t *keys, uint32_t np, KeyLayout L, uint32_t k, uint32_t *seg_start,
                              uint32_t *seg_end) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        uint32_t pr = key_pair(keys[i], L, k);
        if (i == 0 || key_pair(keys[i - 1], L, k) != pr) seg_start[pr] = i;
        if (i + 1 == np || key_pair(keys[i + 1], L, k) != pr) seg_end[pr] = i + 1;
    }
}

struct SegView {
    uint32_t start, len;
    uint64_t base;  // prefix weight before the segment
    const uint64_t *incl;
    __device__ uint64_t excl(uint32_t i) const {  // weight of the first i elements
        return i == 0 ? 0 : incl[start + i - 1] - base;
    }
};

__device__ inline SegView seg_view(const uint32_t *seg_start, const uint32_t *seg_end, uint32_t pr,
                                   const uint64_t *incl) {
    SegView v;
    v.start = seg_start[pr];
    uint32_t end = seg_end[pr];
    v.len = end - v.start;
    v.base = v.start == 0 ? 0 : incl[v.start - 1];
    v.incl = incl;
    return v;
}

// number of i in [0, len) with excl(i) < x (strict) or <= x (non-strict)
__device__ inline uint32_t count_below(const SegView &v, uint64_t x, bool strict) {
    uint32_t lo = 0, hi = v.len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint64_t e = v.excl(mid);
        bool below = strict ? (e < x) : (e <= x);
        if (below) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int64_t floor_div_i64(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

__global__ void k_lp_select(const uint64_t *keys, uint32_t np, KeyLayout L, uint32_t k, const uint32_t *seg_start,
                            const uint32_t *seg_end, const uint64_t *incl, const int64_t *bw, const int64_t *lmax,
                            unsigned long long *best) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        uint64_t key = keys[i];
        uint32_t s = (uint32_t)(key >> L.sh_s) & L.kmask;
        uint32_t t = (uint32_t)(key >> L.sh_t) & L.kmask;
        uint32_t x = s < t ? s : t, y = s < t ? t : s;  // unordered pair, A = moves x->y
        SegView A = seg_view(seg_start, seg_end, x * k + y, incl);
        SegView Bv = seg_view(seg_start, seg_end, y * k + x, incl);
        int64_t beta_x = floor_div_i64(lmax[x] - bw[x], (int64_t)k - 1);
        int64_t beta_y = floor_div_i64(lmax[y] - bw[y], (int64_t)k - 1);
        uint32_t ia, jb;
        if (s == x) {
            uint32_t loc = i - A.start;
            ia = loc + 1;
            jb = count_below(Bv, A.excl(loc), true);
            if (loc == 0 && beta_x >= 0 && beta_y >= 0) atomicMax(&best[x * k + y], 1ull << 32);
        } else {
            uint32_t loc = i - Bv.start;
            jb = loc + 1;
            ia = count_below(A, Bv.excl(loc), false);
            if (loc == 0 && beta_x >= 0 && beta_y >= 0) atomicMax(&best[x * k + y], 1ull << 32);
        }
        int64_t xv = (int64_t)A.excl(ia) - (int64_t)Bv.excl(jb);
        if (-beta_x <= xv && xv <= beta_y)
            atomicMax(&best[x * k + y], ((unsigned long long)(ia + jb + 1) << 32) | ia);
    }
}

// Proposals of the pairs flagged for the device-wide path, from the
// proposal lists (movers of the sub-round are in other pairs).
__global__ __launch_bounds__(BLOCK) void k_collect_slow(const uint32_t *plist, const uint32_t *pcnt,
                                                        uint32_t slot_cap, const uint32_t *part,
                                                        const uint32_t *prop_t, uint32_t k, const uint32_t *slowpair,
                                                        uint32_t *slow, uint32_t *nslow) {
    const uint32_t sl = blockIdx.x % NSLOT, bj = blockIdx.x / NSLOT, nbj = gridDim.x / NSLOT;
    const uint32_t np = pcnt[sl * SPREAD_U32];
    const uint32_t *pl = plist + (size_t)sl * slot_cap;
    for (uint32_t base = bj * BLOCK; base < np; base += nbj * BLOCK) {
        const uint32_t i = base + threadIdx.x;
        bool take = false;
        uint32_t u = 0;
        if (i < np) {
            u = pl[i];
            const uint32_t s = part[u], t = prop_t[u];
            if (s != t) take = slowpair[(s < t ? s : t) * k + (s < t ? t : s)] != 0;
        }
        const uint32_t pos = warp_agg_append(nslow, take);
        if (take) slow[pos] = u;
    }
}

__global__ __launch_bounds__(BLOCK) void k_lp_apply(const uint64_t *keys, const uint32_t *vals, uint32_t np,
                                                    KeyLayout L, uint32_t k, const uint32_t *seg_start,
                                                    const unsigned long long *best, const int32_t *vwgt,
                                                    uint32_t *part, int64_t *bw) {
    __shared__ int64_t dbw[256];
    for (uint32_t b = threadIdx.x; b < k; b += BLOCK) dbw[b] = 0;
    __syncthreads();
    for (uint32_t base = blockIdx.x * BLOCK; base < np; base += gridDim.x * BLOCK) {
        const uint32_t i = base + threadIdx.x;
        bool mv = false;
        if (i < np) {
            uint64_t key = keys[i];
            uint32_t s = (uint32_t)(key >> L.sh_s) & L.kmask;
            uint32_t t = (uint32_t)(key >> L.sh_t) & L.kmask;
            uint32_t x = s < t ? s : t, y = s < t ? t : s;
            unsigned long long bst = best[x * k + y];
            if (bst) {
                uint32_t istar = (uint32_t)bst;
                uint32_t d = (uint32_t)(bst >> 32) - 1;
                uint32_t jstar = d - istar;
                uint32_t loc = i - seg_start[s * k + t];
                mv = (s == x) ? (loc < istar) : (loc < jstar);
            }
            if (mv) {
                const uint32_t u = vals[i];
                part[u] = t;
                int64_t c = vwgt[u];
                atomicAdd((unsigned long long *)&dbw[s], (unsigned long long)(-c));
                atomicAdd((unsigned long long *)&dbw[t], (unsigned long long)c);
            }
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < k; b += BLOCK)
        if (dbw[b]) atomic_add_i64(&bw[b], dbw[b]);
}

// ---------------------------------------------------------------------------
// Whole-pair fast path.  The two-pointer walk of a block pair ends in the
// state that takes every move of both directions; being the last state
// visited, it is the selected one whenever it is feasible.  So if
// -beta_x <= w(M_xy) - w(M_yx) <= beta_y all moves of the pair are applied at
// once, in any order, and only the remaining pairs need the sorted walk.
// Block-weight changes go to dbw_g so that the sorted walk still reads the
// snapshot block weights.  Movers are not listed: a proposer has moved iff
// its block is now its proposed target.  The proposals of the other pairs go
// to their pair's segment of `seg`: every unordered pair {x < y} owns
// seg_cap slots (a pair of more proposals goes to the device-wide path,
// which collects them again from the proposal lists).
// Workgroup b reads proposal list b % NSLOT (the grid is a multiple of NSLOT).
// ---------------------------------------------------------------------------
__device__ inline size_t pair_segment(uint32_t x, uint32_t y, uint32_t k, uint32_t seg_cap) {
    return ((size_t)x * (2 * k - x - 1) / 2 + (y - x - 1)) * seg_cap;  // triangular index of {x < y}
}

__global__ __launch_bounds__(BLOCK) void k_lp_fast(const uint32_t *plist, const uint32_t *pcnt, uint32_t slot_cap,
                                                   const uint32_t *prop_t, const uint32_t *pw, uint32_t k,
                                                   const int32_t *vwgt, uint32_t *part, const int64_t *bw,
                                                   const int64_t *lmax, int64_t *dbw_g, uint32_t *pcur, uint32_t *seg,
                                                   uint32_t seg_cap, uint32_t *spairs, uint32_t *nsp, LpCtl ctl) {
    if (lp_skip(ctl)) return;
    constexpr uint32_t HSLOTS = 2 * BLOCK;  // pair table of one step: at most BLOCK keys, half full
    static_assert(HSLOTS == 512, "the slot hash takes 9 bits");
    __shared__ int64_t dbw[256];
    __shared__ uint32_t hkey[HSLOTS], hcnt[HSLOTS], hbase[HSLOTS];
    for (uint32_t b = threadIdx.x; b < k; b += BLOCK) dbw[b] = 0;
    __syncthreads();
    const uint32_t sl = blockIdx.x % NSLOT, bj = blockIdx.x / NSLOT, nbj = gridDim.x / NSLOT;
    const uint32_t np = pcnt[sl * SPREAD_U32];
    const uint32_t *pl = plist + (size_t)sl * slot_cap;
    for (uint32_t base = bj * BLOCK; base < np; base += nbj * BLOCK) {  // uniform per block
        const uint32_t i = base + threadIdx.x;
        bool slow = false;
        uint32_t u = 0, x = 0, y = 0;
        if (i < np) {
            u = pl[i];
            const uint32_t s = part[u], t = prop_t[u];
            x = s < t ? s : t;
            y = s < t ? t : s;
            const int64_t xf = (int64_t)pw[x * k + y] - (int64_t)pw[y * k + x];
            const int64_t beta_x = floor_div_i64(lmax[x] - bw[x], (int64_t)k - 1);
            const int64_t beta_y = floor_div_i64(lmax[y] - bw[y], (int64_t)k - 1);
            if (-beta_x <= xf && xf <= beta_y) {
                part[u] = t;
                int64_t c = vwgt[u];
                atomicAdd((unsigned long long *)&dbw[s], (unsigned long long)(-c));
                atomicAdd((unsigned long long *)&dbw[t], (unsigned long long)c);
            } else {
                slow = true;
            }
        }
        // The step's proposals of oversized pairs take their segment positions
        // with one global atomic per pair and step: an LDS table counts them
        // per pair first (a pair whose proposals all hit one global counter
        // would serialise them).  The order inside a segment does not
        // matter: the pair kernel sorts it.
        if (__syncthreads_or(slow)) {
            for (uint32_t q = threadIdx.x; q < HSLOTS; q += BLOCK) { hkey[q] = NONE; hcnt[q] = 0; }
            __syncthreads();
            const uint32_t key = x * k + y;
            uint32_t slot = 0, rank = 0;
            if (slow) {
                slot = (key * 2654435761u) >> (32 - 9);  // 9 bits: HSLOTS = 512
                for (;;) {
                    const uint32_t old = atomicCAS(&hkey[slot], NONE, key);
                    if (old == NONE || old == key) break;
                    slot = (slot + 1) & (HSLOTS - 1);
                }
                rank = atomicAdd(&hcnt[slot], 1u);
            }
            __syncthreads();
            if (slow && rank == 0) hbase[slot] = atomicAdd(&pcur[key], hcnt[slot]);
            __syncthreads();
            if (slow) {
                const uint32_t at = hbase[slot] + rank;
                if (at < seg_cap) seg[pair_segment(x, y, k, seg_cap) + at] = u;
                if (at == 0) spairs[atomicAdd(nsp, 1u)] = key;  // the pair's first proposal lists it
            }
            __syncthreads();  // the table is cleared by the next step
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < k; b += BLOCK)
        if (dbw[b]) atomic_add_i64(&dbw_g[b], dbw[b]);
}

// Block weight limits: every block `uniform`, or blocks 0 and 1 `l0`, `l1`
// (a bisection, k = 2).
__global__ void k_set_limits(int64_t *lmax, uint32_t k, int64_t uniform, int64_t l0, int64_t l1) {
    for (uint32_t b = threadIdx.x; b < k; b += blockDim.x) lmax[b] = k == 2 ? (b == 0 ? l0 : l1) : uniform;
}

// Clears up to ZERO_MAX word ranges in one launch.
constexpr int ZERO_MAX = 12;
struct ZeroSet {
    uint32_t *p[ZERO_MAX];
    size_t len[ZERO_MAX];
    int n;
    void add(void *q, size_t words) {
        if (words) { p[n] = (uint32_t *)q; len[n] = words; ++n; }
    }
};
__global__ void k_zero_words(ZeroSet z) {
    for (int a = 0; a < z.n; ++a)
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.len[a];
             i += (size_t)gridDim.x * blockDim.x)
            z.p[a][i] = 0;
}

__global__ void k_add_dbw(int64_t *bw, int64_t *dbw_g, uint32_t k) {
    for (uint32_t b = threadIdx.x; b < k; b += blockDim.x)
        if (dbw_g[b]) { bw[b] += dbw_g[b]; dbw_g[b] = 0; }
}

// Total of the spread objective accumulator (one wave).
__global__ void k_objective_total(const int64_t *f, int64_t *out) {
    const int64_t t = spread_total_wave(f);
    if (threadIdx.x == 0) *out = t;
}

// Largest proposed gain of the device-wide path's proposals.
__global__ __launch_bounds__(BLOCK) void k_gain_max(const uint32_t *list, uint32_t cnt, const uint32_t *prop_g,
                                                    uint32_t *out) {
    __shared__ uint32_t red[BLOCK / WAVE];
    uint32_t mx = 0;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < cnt; i += gridDim.x * BLOCK) {
        const uint32_t g = prop_g[list[i]];
        mx = g > mx ? g : mx;
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
        if (mx) atomicMax(out, mx);
    }
}

// ---------------------------------------------------------------------------
// Pairs whose whole move sets do not fit: one workgroup per block pair.
//   k_lp_fast    puts the proposals of every pair that fails the whole-pair
//                test into the pair's segment, in no particular order, and
//                lists the pair.
//   k_lp_pairs   takes the listed pairs, sorts each segment in
//                LDS by (direction, gain desc, u asc) -- a total order, so the
//                arbitrary segment order does not matter -- walks the merge
//                path of the pair and applies the approved prefixes.  A pair
//                of more than PAIR_MAX proposals is handed to the device-wide
//                path: it is flagged and the abort word records the
//                sub-round, after which the host collects the flagged pairs'
//                proposals, finishes the sub-round and replays the rest of
//                the round.
// Block-weight changes go to dbw_g; every test of the sub-round reads the
// snapshot block weights.
// ---------------------------------------------------------------------------
constexpr int PAIR_THREADS = 512;
constexpr uint32_t PAIR_MAX = 4096;

// Merge-path view of one direction of a pair: element i of the direction is
// sorted position start + i; excl(i) is the weight of its first i elements.
struct LSeg {
    uint32_t start, len;
    uint32_t base;
    const uint32_t *incl;
    __device__ uint32_t excl(uint32_t i) const { return i == 0 ? 0u : incl[start + i - 1] - base; }
};

__device__ inline uint32_t lcount_below(const LSeg &v, uint32_t x, bool strict) {
    uint32_t lo = 0, hi = v.len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t e = v.excl(mid);
        bool below = strict ? (e < x) : (e <= x);
        if (below) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(PAIR_THREADS) void k_lp_pairs(const uint32_t *spairs, const uint32_t *nsp,
                                                           const uint32_t *pc, const uint32_t *seg, uint32_t seg_cap,
                                                           uint32_t k,
                                                           const uint32_t *prop_g, const int32_t *vwgt,
                                                           uint32_t *part, const int64_t *bw, const int64_t *lmax,
                                                           int64_t *dbw_g, uint32_t *slowpair, LpCtl ctl) {
    __shared__ uint64_t skey[PAIR_MAX];
    __shared__ uint32_t sincl[PAIR_MAX];
    __shared__ uint32_t wsum[PAIR_THREADS / WAVE];
    __shared__ unsigned long long sbest;
    // an earlier sub-round was cut short (a block of this launch may raise
    // the word for this sub-round: that does not stop the others)
    const uint32_t aw = *ctl.abort;
    if ((aw && aw != ctl.stamp) || (ctl.prev && *ctl.prev == 0)) return;
    const uint32_t tid = threadIdx.x;
    const uint32_t np = *nsp;
    for (uint32_t q = blockIdx.x; q < np; q += gridDim.x) {
        const uint32_t pi = spairs[q];
        const uint32_t x = pi / k, y = pi % k;  // x < y
        const uint32_t nA = pc[pi], L = nA + pc[y * k + x];
        if (L > PAIR_MAX || L > seg_cap) {  // uniform per block
            if (tid == 0) {
                slowpair[pi] = 1;
                atomicExch(ctl.abort, ctl.stamp);
            }
            continue;
        }
        const uint32_t *sg = seg + pair_segment(x, y, k, seg_cap);
        uint32_t n2 = 1;
        while (n2 < L) n2 <<= 1;
        // key: direction (0: x -> y), then gain descending, then u (< 2^31)
        for (uint32_t i = tid; i < n2; i += PAIR_THREADS) {
            uint64_t key = ~0ull;
            if (i < L) {
                const uint32_t u = sg[i];
                const uint64_t dir = part[u] == x ? 0ull : 1ull;
                key = (dir << 63) | ((uint64_t)(0xFFFFFFFFu - prop_g[u]) << 31) | (uint64_t)u;
            }
            skey[i] = key;
        }
        if (tid == 0) sbest = 0;
        __syncthreads();
        for (uint32_t kk = 2; kk <= n2; kk <<= 1) {
            for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < n2; i += PAIR_THREADS) {
                    const uint32_t l = i ^ j;
                    if (l > i) {
                        const uint64_t a = skey[i], b = skey[l];
                        if ((a > b) == ((i & kk) == 0)) { skey[i] = b; skey[l] = a; }
                    }
                }
                __syncthreads();
            }
        }
        // inclusive prefix of vertex weights in sorted order (c(V) < 2^31)
        uint32_t carry = 0;
        for (uint32_t c0 = 0; c0 < L; c0 += PAIR_THREADS) {
            const uint32_t i = c0 + tid;
            const uint32_t w = i < L ? (uint32_t)vwgt[(uint32_t)(skey[i] & 0x7FFFFFFFu)] : 0u;
            uint32_t tot;
            const uint32_t incl = block_incl_scan_n<uint32_t, PAIR_THREADS>(w, wsum, &tot);
            if (i < L) sincl[i] = carry + incl;
            carry += tot;
        }
        __syncthreads();
        LSeg A, Bv;
        A.start = 0; A.len = nA; A.base = 0; A.incl = sincl;
        Bv.start = nA; Bv.len = L - nA; Bv.base = nA ? sincl[nA - 1] : 0u; Bv.incl = sincl;
        const int64_t beta_x = floor_div_i64(lmax[x] - bw[x], (int64_t)k - 1);
        const int64_t beta_y = floor_div_i64(lmax[y] - bw[y], (int64_t)k - 1);
        if (tid == 0 && beta_x >= 0 && beta_y >= 0) atomicMax(&sbest, 1ull << 32);  // the start state
        // every element tests the walk state right after it
        for (uint32_t i = tid; i < L; i += PAIR_THREADS) {
            uint32_t ia, jb;
            if (i < nA) {
                ia = i + 1;
                jb = lcount_below(Bv, A.excl(i), true);
            } else {
                jb = i - nA + 1;
                ia = lcount_below(A, Bv.excl(i - nA), false);
            }
            const int64_t xv = (int64_t)A.excl(ia) - (int64_t)Bv.excl(jb);
            if (-beta_x <= xv && xv <= beta_y) atomicMax(&sbest, ((unsigned long long)(ia + jb + 1) << 32) | ia);
        }
        __syncthreads();
        const unsigned long long bst = sbest;
        uint32_t istar = 0, jstar = 0;
        if (bst) {
            istar = (uint32_t)bst;
            jstar = (uint32_t)(bst >> 32) - 1 - istar;
        }
        for (uint32_t i = tid; i < L; i += PAIR_THREADS)
            if (i < nA ? i < istar : i - nA < jstar) part[(uint32_t)(skey[i] & 0x7FFFFFFFu)] = i < nA ? y : x;
        if (tid == 0 && bst) {
            const int64_t wa = A.excl(istar), wb = Bv.excl(jstar);
            if (wa != wb) {
                atomic_add_i64(&dbw_g[x], wb - wa);
                atomic_add_i64(&dbw_g[y], wa - wb);
            }
        }
        __syncthreads();  // the arrays are reused by the next pair
    }
}

// Measurement only: compulsory bytes of one update launch (mover list and
// incidence lists; for every distinct touched net its stamp, offsets, pins,
// their blocks, weight, old Lambda and new Lambda / Lambda1).
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_account_update(const uint32_t *pin_off, const uint32_t *inc_off,
                                                          const uint32_t *inc, const uint32_t *plist,
                                                          const uint32_t *pcnt, uint32_t slot_cap,
                                                          const uint32_t *part, const uint32_t *prop_t,
                                                          uint32_t *nmark, uint32_t stamp, unsigned long long *acc,
                                                          LpCtl ctl) {
    __shared__ unsigned long long red[BLOCK / WAVE];
    if (lp_skip(ctl)) return;  // the sub-round does nothing
    unsigned long long bytes = 0;
    const uint32_t sl = blockIdx.x % NSLOT, bj = blockIdx.x / NSLOT, nbj = gridDim.x / NSLOT;
    const uint32_t cnt = pcnt[sl * SPREAD_U32];
    const uint32_t *pl = plist + (size_t)sl * slot_cap;
    for (uint32_t idx = bj * blockDim.x + threadIdx.x; idx < cnt; idx += nbj * blockDim.x) {
        const uint32_t u = pl[idx];
        bytes += 4 + 4 + 4;  // proposal entry, block, target
        if (part[u] != prop_t[u]) continue;
        const uint32_t j0 = inc_off[u], j1 = inc_off[u + 1];
        bytes += 8 + 4ull * (j1 - j0);
        for (uint32_t j = j0; j < j1; ++j) {
            const uint32_t e = inc[j];
            if (atomicExch(&nmark[e], stamp) == stamp) continue;
            const uint32_t len = pin_off[e + 1] - pin_off[e];
            bytes += 8 + 8 + 8ull * len + 4 + 24ull * KW;
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

// Recomputes net e once per sub-round (the first caller to stamp it owns
// it): Lambda / Lambda1 from the pins' blocks, boundary counts of its pins on
// a cut flip; nets of more than 64 pins go to the long-net list.  Returns the
// objective change w(e) (max(lambda'-1,0) - max(lambda-1,0)).
// Graph levels keep no net records: the cut bit of every edge (the bitmap
// the connectivity kernel leaves) is the state, and an edge's update
// compares it with its endpoints' blocks now.  cut == nullptr on hypergraph
// levels.
struct GraphUpd {
    const int32_t *nwgt;
    uint32_t *cut;
};

template <int KW>
__device__ inline int64_t update_net(const uint32_t *pin_off, const uint32_t *pins, uint32_t e, const uint32_t *part,
                                     NetRec<KW> *nr, uint32_t *tstamp, uint32_t stamp, uint32_t *longl,
                                     uint32_t *nlong, uint32_t *bcnt, const GraphUpd &gu) {
    if (atomicExch(&tstamp[e], stamp) == stamp) return 0;
    if (gu.cut) {
        const uint32_t x = pins[2 * (size_t)e], y = pins[2 * (size_t)e + 1];
        const bool now = part[x] != part[y];
        const bool was = (gu.cut[e >> 5] >> (e & 31)) & 1u;
        if (now == was) return 0;
        atomicXor(&gu.cut[e >> 5], 1u << (e & 31));
        const uint32_t delta = now ? 1u : 0xFFFFFFFFu;
        atomicAdd(&bcnt[x], delta);
        atomicAdd(&bcnt[y], delta);
        return now ? (int64_t)gu.nwgt[e] : -(int64_t)gu.nwgt[e];
    }
    const uint32_t b = pin_off[e], len = pin_off[e + 1] - b;
    if (len > 64) {
        longl[atomicAdd(nlong, 1u)] = e;
        return 0;
    }
    uint64_t once[KW], twice[KW];
    net_bits<KW>(pins, b, len, part, once, twice);
    NetRec<KW> &R = nr[e];
    const int lnew = popc_bits<KW>(once), lold = popc_bits<KW>(R.lam);
    const int64_t d = lam_cost(lnew) - lam_cost(lold);
#pragma unroll
    for (int q = 0; q < KW; ++q) {
        R.lam[q] = once[q];
        R.lam1[q] = once[q] & ~twice[q];
    }
    if ((lnew > 1) != (lold > 1)) {  // cut status flipped: boundary counts of its pins
        const uint32_t delta = lnew > 1 ? 1u : 0xFFFFFFFFu;
        for (uint32_t q = b; q < b + len; ++q) atomicAdd(&bcnt[pins[q]], delta);
    }
    return d * R.w;
}

// Movers of more than HUB_DEG nets: their incidence lists are cut into chunks
// of BLOCK nets spread over the whole grid (a net per thread).
// The listed movers' incidence lists are cut into chunks of ADJ_CHUNK nets
// (cbase from k_heavy_chunks), so the grid is balanced whatever the degrees.
template <int KW>
__global__ __launch_bounds__(BLOCK) void k_lp_update_heavy(const uint32_t *pin_off, const uint32_t *pins,
                                                           const uint32_t *inc_off, const uint32_t *inc,
                                                           const uint32_t *heavy, const uint32_t *nheavy,
                                                           const uint32_t *cbase, const uint32_t *part,
                                                           NetRec<KW> *nr, uint32_t *tstamp, uint32_t stamp,
                                                           int64_t *f, uint32_t *longl, uint32_t *nlong,
                                                           uint32_t *bcnt, LpCtl ctl, GraphUpd gu) {
    if (lp_skip(ctl)) return;
    __shared__ int64_t red[BLOCK / WAVE];
    const uint32_t cnt = *nheavy, total = cbase[cnt];
    int64_t acc = 0;
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
        uint32_t lo = 0, hi = cnt;  // the listed mover whose chunks hold g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (cbase[mid] <= g) lo = mid; else hi = mid;
        }
        const uint32_t u = heavy[lo], j1 = inc_off[u + 1];
        const uint32_t jb = inc_off[u] + (g - cbase[lo]) * ADJ_CHUNK, je = jb + ADJ_CHUNK < j1 ? jb + ADJ_CHUNK : j1;
        for (uint32_t j = jb + threadIdx.x; j < je; j += BLOCK)
            acc += update_net<KW>(pin_off, pins, inc[j], part, nr, tstamp, stamp, longl, nlong, bcnt, gu);
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
        if (t) spread_add_i64(f, t);
    }
}

// Lambda / Lambda1 of every net of a moved node, recomputed once: G lanes per
// mover; the first lane to stamp a net in this sub-round owns it.  Nets of
// more than 64 pins are forwarded to the wave kernel.  The objective changes
// by w(e) (max(lambda'-1,0) - max(lambda-1,0)); the sub-round's move count is
// added to the round's.
// State the next sub-round's gains start from: its proposal counters and pair
// sums at zero, and this sub-round's block-weight changes in the block
// weights.  Cleared by the last kernel of a sub-round that every sub-round
// runs (the update), after every reader.
// The proposal-list lengths come in two sets used by alternate sub-rounds:
// the update reads its own sub-round's set and clears the other one.
struct NextSub {
    uint32_t *scal, *pw, *pc, *pcur, *ccnt;
    uint32_t kk, k;
    int64_t *bw, *dbw_g;
    uint32_t *pcnt_next;
};
__device__ inline void next_subround(const NextSub &z) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    if (tid == 0) { z.scal[25] = 0; z.scal[26] = 0; }  // listed pairs, hub candidates
    if (tid < NSLOT) z.pcnt_next[tid * SPREAD_U32] = 0;
    if (tid < 3 * NSLOT) z.ccnt[tid * SPREAD_U32] = 0;  // candidate lists (read by this sub-round's gains only)
    for (uint32_t i = tid; i < z.kk; i += nt) { z.pw[i] = 0; z.pc[i] = 0; z.pcur[i] = 0; }
    if (blockIdx.x == 0)
        for (uint32_t b = threadIdx.x; b < z.k; b += blockDim.x) {
            const int64_t d = z.dbw_g[b];
            if (d) { z.bw[b] += d; z.dbw_g[b] = 0; }
        }
}

// The movers are the proposers now in their target block; workgroup b reads
// proposal list b % NSLOT (the grid is a multiple of NSLOT).  `moves` is set
// when the sub-round moved a node.
template <int KW, int G>
__global__ __launch_bounds__(BLOCK) void k_lp_update_movers(const uint32_t *pin_off, const uint32_t *pins,
                                                            const uint32_t *inc_off, const uint32_t *inc,
                                                            const uint32_t *plist, const uint32_t *pcnt,
                                                            uint32_t slot_cap, const uint32_t *prop_t,
                                                            const uint32_t *part, NetRec<KW> *nr, uint32_t *tstamp,
                                                            uint32_t stamp, int64_t *f, uint32_t *longl,
                                                            uint32_t *nlong, uint32_t *moves, uint32_t *bcnt,
                                                            uint32_t *heavy, uint32_t *nheavy, NextSub z,
                                                            LpCtl ctl, GraphUpd gu) {
    if (lp_skip(ctl)) return;
    next_subround(z);
    __shared__ int64_t red[BLOCK / WAVE];
    __shared__ uint32_t moved_any;
    constexpr int GPB = BLOCK / G;
    const uint32_t sl = blockIdx.x % NSLOT, bj = blockIdx.x / NSLOT, nbj = gridDim.x / NSLOT;
    const uint32_t cnt = pcnt[sl * SPREAD_U32];
    const uint32_t *pl = plist + (size_t)sl * slot_cap;
    if (threadIdx.x == 0) moved_any = 0;
    __syncthreads();
    const uint32_t g = threadIdx.x / G, l = threadIdx.x % G;
    int64_t acc = 0;
    bool moved = false;
    for (uint32_t idx = bj * GPB + g; idx < cnt; idx += nbj * GPB) {
        const uint32_t u = pl[idx];
        if (part[u] != prop_t[u]) continue;  // proposed but not moved (uniform per group)
        moved = true;
        const uint32_t j0 = inc_off[u], j1 = inc_off[u + 1];
        if (j1 - j0 > HUB_DEG) {  // uniform per group: left to the chunked kernel
            if (l == 0) heavy[atomicAdd(nheavy, 1u)] = u;
            continue;
        }
        for (uint32_t j = j0 + l; j < j1; j += G)
            acc += update_net<KW>(pin_off, pins, inc[j], part, nr, tstamp, stamp, longl, nlong, bcnt, gu);
    }
    acc = wave_sum(acc);
    if (moved) moved_any = 1u;
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
        if (t) spread_add_i64(f, t);
        if (moved_any) *moves = 1u;  // a plain store: only ever set to 1
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct RefineBufs {
    void *nr;  // NetRec<KW>[m]
    int64_t *f;     // objective, spread over SPREAD slots
    int64_t *bw;
    uint32_t *longl, *plist, *prop_t, *prop_g, *tstamp, *bcnt, *scal, *heavy, *hcbase, *pw, *slow;
    int64_t *lmaxv;  // [k] block weight limits
    uint32_t *pcnt;  // [2][NSLOT * SPREAD_U32] proposal-list lengths, alternate sub-rounds
    uint32_t *cl;    // [3][NSLOT] candidate lists by degree class and slot
    uint32_t *ccnt;  // [3 * NSLOT * SPREAD_U32] their lengths
    uint32_t *dlists;  // hub candidates of the sub-round
    uint32_t *pc, *pcur, *seg;  // per-pair proposal counts, appends and segments of over-budget pairs
    uint32_t *spairs;           // the sub-round's over-budget pairs
    uint32_t *slowpair;         // [k*k] pairs handed to the device-wide path
    uint32_t *rmoves;           // [LP_MAX_ROUNDS] moves flag of every round
    uint64_t *cut;              // [ceil(m / 64)] cut bit of every net, for the boundary counts
    int64_t *dbw_g;
    uint64_t *keys, *keys_alt, *incl;
    uint32_t *vals, *vals_alt, *seg_start, *seg_end;
    unsigned long long *best;
};

constexpr uint32_t LP_MAX_ROUNDS = 65536;  // above the largest accepted R_lp
constexpr uint32_t LP_ROUND_BATCH = 8;      // rounds queued per host read-back

// Slots per unordered block pair for the sorted walk's proposals.
static uint32_t pair_seg_cap(uint32_t n) { return n < PAIR_MAX ? n : PAIR_MAX; }

static void plan(Arena &A, uint32_t n, uint32_t m, uint32_t k, RefineBufs &B) {
    int KW = (int)((k + 63) / 64);
    B.nr = A.alloc<char>((size_t)m * netrec_bytes(KW));
    B.f = A.alloc<int64_t>((size_t)SPREAD * SPREAD_I64);
    B.pcnt = A.alloc<uint32_t>((size_t)2 * NSLOT * SPREAD_U32);
    B.cl = A.alloc<uint32_t>(3 * ((size_t)n + (size_t)(3 * NSLOT) * GAIN_CH));
    B.ccnt = A.alloc<uint32_t>((size_t)3 * NSLOT * SPREAD_U32);
    B.bw = A.alloc<int64_t>(k);
    B.longl = A.alloc<uint32_t>(m);
    B.dlists = A.alloc<uint32_t>(n);
    B.bcnt = A.alloc<uint32_t>(n);
    B.plist = A.alloc<uint32_t>((size_t)n + (size_t)(3 * NSLOT) * GAIN_CH);  // NSLOT lists of slot_cap (chunk_slot_cap)
    B.prop_t = A.alloc<uint32_t>(n);
    B.prop_g = A.alloc<uint32_t>(n);
    B.tstamp = A.alloc<uint32_t>(m);
    B.scal = A.alloc<uint32_t>(32);
    B.keys = A.alloc<uint64_t>(n);
    B.keys_alt = A.alloc<uint64_t>(n);
    B.incl = A.alloc<uint64_t>(n);
    B.vals = A.alloc<uint32_t>(n);
    B.vals_alt = A.alloc<uint32_t>(n);
    B.seg_start = A.alloc<uint32_t>((size_t)k * k);
    B.seg_end = A.alloc<uint32_t>((size_t)k * k);
    B.best = A.alloc<unsigned long long>((size_t)k * k);
    B.pw = A.alloc<uint32_t>((size_t)k * k);
    B.pc = A.alloc<uint32_t>((size_t)k * k);
    B.pcur = A.alloc<uint32_t>((size_t)k * k);
    B.slowpair = A.alloc<uint32_t>((size_t)k * k);
    B.spairs = A.alloc<uint32_t>((size_t)k * k);
    B.rmoves = A.alloc<uint32_t>(LP_MAX_ROUNDS);
    B.cut = A.alloc<uint64_t>(((size_t)m + WAVE - 1) / WAVE);
    B.seg = A.alloc<uint32_t>((size_t)k * (k - 1) / 2 * pair_seg_cap(n));
    B.slow = A.alloc<uint32_t>(n);
    B.heavy = A.alloc<uint32_t>(n);
    B.lmaxv = A.alloc<int64_t>(k);
    B.hcbase = A.alloc<uint32_t>((size_t)n + 1);
    B.dbw_g = A.alloc<int64_t>(k);
    sort_reserve(A, n);
    scan_reserve<uint64_t>(A, n);
}

size_t refine_workspace(uint32_t n, uint32_t m, uint32_t k) {
    Arena A(nullptr, 0);
    RefineBufs B;
    plan(A, n, m, k, B);
    return A.peak;
}

// Net records and objective of `part`; the objective slots and the long-net
// count start at zero (cleared here unless the caller has).
template <int KW>
static void build_conn(const hgp_hg &h, const uint32_t *part, RefineBufs &B, hipStream_t st, bool zeroed = false) {
    if (!zeroed) {
        HGP_CHECK_HIP(hipMemsetAsync(B.f, 0, sizeof(int64_t) * SPREAD * SPREAD_I64, st));
        HGP_CHECK_HIP(hipMemsetAsync(B.scal + 12, 0, sizeof(uint32_t), st));
    }
    if (h.m) {
        k_conn_small<KW><<<grid_for(h.m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
            h.pin_off, h.pins, h.m, h.nwgt, part, (NetRec<KW> *)B.nr, B.f, B.longl, B.scal + 12, B.cut);
        HGP_LAUNCH_CHECK();
        k_conn_long<KW><<<FILL_BLOCKS / 4, BLOCK, 0, st>>>(h.pin_off, h.pins, B.longl, B.scal + 12, h.nwgt, part,
                                                           (NetRec<KW> *)B.nr, B.f, false, nullptr,
                                                           LpCtl{nullptr, nullptr, 0}, (uint32_t *)B.cut);
        HGP_LAUNCH_CHECK();
    }
}

static void block_weights(const uint32_t *part, const int32_t *vwgt, uint32_t n, uint32_t k, int64_t *bw,
                          hipStream_t st) {
    HGP_CHECK_HIP(hipMemsetAsync(bw, 0, sizeof(int64_t) * k, st));
    k_block_weights<<<grid_for(n, BLOCK * 8, REDUCE_BLOCKS), BLOCK, 0, st>>>(part, vwgt, n, k, bw);
    HGP_LAUNCH_CHECK();
}

template <int KW>
static void objective_t(const hgp_hg &h, uint32_t k, const uint32_t *part, int64_t *obj, int64_t *bw_out, Arena &A,
                        hipStream_t st) {
    size_t mk = A.mark();
    RefineBufs B;
    plan(A, h.n, h.m, k, B);
    build_conn<KW>(h, part, B, st);
    k_objective_total<<<1, WAVE, 0, st>>>(B.f, obj);
    HGP_LAUNCH_CHECK();
    if (bw_out) block_weights(part, h.vwgt, h.n, k, bw_out, st);
    stream_sync(st);
    A.release(mk);
}

void objective(const hgp_hg &h, uint32_t k, const uint32_t *part, int64_t *obj, int64_t *bw, Arena &A,
               hipStream_t st) {
    switch ((k + 63) / 64) {
        case 1: objective_t<1>(h, k, part, obj, bw, A, st); break;
        case 2: objective_t<2>(h, k, part, obj, bw, A, st); break;
        case 3: objective_t<3>(h, k, part, obj, bw, A, st); break;
        default: objective_t<4>(h, k, part, obj, bw, A, st); break;
    }
}

template <int KW>
static void refine_t(const hgp_hg &h, const hgp_params &prm, uint32_t level, uint32_t *part, int64_t *obj,
                     int64_t *bw_out, Arena &A, hipStream_t st, int64_t W_known, uint32_t *rounds_out,
                     const int64_t *side_limits) {
    const uint32_t n = h.n, m = h.m, k = prm.k;
    size_t mk = A.mark();
    RefineBufs B;
    plan(A, n, m, k, B);
    const int64_t W = W_known >= 0 ? W_known : total_weight(h.vwgt, n, A, st);
    // the weight limit of every block: L_max = (1 + eps) ceil(c(V) / k), or
    // the two side limits of a bisection of the recursive bipartitioning
    const int64_t Lmax = ((int64_t)(prm.eps_den + prm.eps_num) * ((W + k - 1) / k)) / (int64_t)prm.eps_den;
    k_set_limits<<<1, 256, 0, st>>>(B.lmaxv, k, Lmax, side_limits ? side_limits[0] : Lmax,
                                    side_limits ? side_limits[1] : Lmax);
    HGP_LAUNCH_CHECK();
    const int64_t *lmax = B.lmaxv;
    const uint64_t mseed = mix64(prm.seed);
    // device scalars: ntouched and nlong are adjacent so one memset clears both
    uint32_t *gmax = B.scal + 1, *ntouched = B.scal + 2, *nlong = B.scal + 3,
             *dcnt = B.scal + 5 /* [NDEG] */, *nheavy = B.scal + 24,
             *nslow = B.scal + 13;

    {  // every counter, flag, stamp and accumulator of the level starts at zero
        ZeroSet z{};
        z.add(B.scal, 32);
        z.add(B.pw, (size_t)k * k);
        z.add(B.pc, (size_t)k * k);
        z.add(B.pcur, (size_t)k * k);
        z.add(B.slowpair, (size_t)k * k);
        z.add(B.dbw_g, 2 * (size_t)k);
        z.add(B.bw, 2 * (size_t)k);
        z.add(B.pcnt, 2 * NSLOT * SPREAD_U32);
        z.add(B.rmoves, std::min<uint32_t>(prm.lp_rounds, LP_MAX_ROUNDS));
        z.add(B.f, 2 * SPREAD * SPREAD_I64);
        z.add(B.tstamp, m);
        z.add(B.ccnt, 3 * NSLOT * SPREAD_U32);
        k_zero_words<<<grid_for(std::max<size_t>(m, (size_t)k * k), BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(z);
        HGP_LAUNCH_CHECK();
    }
    // degree classes of the nodes (lanes per node 1 / 8 / 64) and the largest net
    k_deg_classify<<<grid_for(n, BLOCK, REDUCE_BLOCKS), BLOCK, 0, st>>>(h.inc_off, n, dcnt);
    HGP_LAUNCH_CHECK();
    if (h.m) {
        k_max_net<<<grid_for(h.m, BLOCK, REDUCE_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.m, B.scal + 4);
        HGP_LAUNCH_CHECK();
    }
    uint32_t dc[NDEG], hs[16];
    read_back(hs, B.scal, sizeof(hs), st, false);
    for (int c = 0; c < NDEG; ++c) dc[c] = hs[5 + c];
    const bool long_nets = hs[4] > 64;  // nets of more than 64 pins exist on this level
    // A graph level (every net has two pins) keeps no net records: the
    // adjacency array (built here when the workspace has room for it) and the
    // cut bits stand in for them.
    GraphUpd gupd{h.nwgt, nullptr};
    const uint32_t *adj = nullptr;
    const int32_t *adjw = nullptr;
    if (h.m && hs[4] == 2 && (uint64_t)h.p == 2ull * h.m &&
        A.remaining() >= 8ull * h.p + 4ull * n + 2048) {
        uint32_t *ad = A.alloc<uint32_t>(h.p);
        int32_t *aw = A.alloc<int32_t>(h.p);
        uint32_t *cbase = A.alloc<uint32_t>((size_t)n + 1);
        uint32_t *nheavy_adj = B.scal + 27;  // cleared with the level's scalars
        k_graph_adj<<<grid_for(n, BLOCK, 4 * FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, h.inc, h.pin_off, h.pins,
                                                                          h.nwgt, n, ad, aw, B.heavy, nheavy_adj);
        HGP_LAUNCH_CHECK();
        k_heavy_chunks<<<1, HEAVY_SCAN, 0, st>>>(h.inc_off, B.heavy, nheavy_adj, cbase);
        HGP_LAUNCH_CHECK();
        k_graph_adj_heavy<<<FILL_BLOCKS, BLOCK, 0, st>>>(h.inc_off, h.inc, h.pin_off, h.pins, h.nwgt, B.heavy,
                                                        nheavy_adj, cbase, ad, aw);
        HGP_LAUNCH_CHECK();
        k_conn_graph<<<grid_for(h.m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, h.m, h.nwgt, part,
                                                                          B.f, B.cut);
        HGP_LAUNCH_CHECK();
        adj = ad;
        adjw = aw;
        gupd.cut = (uint32_t *)B.cut;
    } else {
        build_conn<KW>(h, part, B, st, true);
    }
    k_block_weights<<<grid_for(n, BLOCK * 8, REDUCE_BLOCKS), BLOCK, 0, st>>>(part, h.vwgt, n, k, B.bw);
    HGP_LAUNCH_CHECK();
    if ((uint64_t)h.p >= (uint64_t)16 * n)  // average degree of at least 16: a wave per node
        k_init_bcnt_wave<KW><<<grid_for((size_t)n * WAVE, BLOCK, 4 * FILL_BLOCKS), BLOCK, 0, st>>>(
            h.inc_off, h.inc, n, (const uint32_t *)B.cut, B.bcnt, B.heavy, B.scal + 28);
    else
        k_init_bcnt<KW><<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, h.inc, n,
                                                                           (const uint32_t *)B.cut, B.bcnt);
    HGP_LAUNCH_CHECK();
    if ((uint64_t)h.p >= (uint64_t)16 * n && (uint64_t)h.p > BCNT_HUGE) {  // listed hubs of the wave kernel
        k_init_bcnt_huge<<<256, BCNT_HUGE_THREADS, 0, st>>>(h.inc_off, h.inc, (const uint32_t *)B.cut, B.heavy,
                                                            B.scal + 28, B.bcnt);
        HGP_LAUNCH_CHECK();
    }
    const uint32_t S = prm.lp_subrounds;
    // gains: chunks of `gch` vertices (a power of two in [64, GAIN_CH], about
    // n / 1024, so that even small levels spread over many workgroups)
    uint32_t gch = 64;
    while (gch < GAIN_CH && (size_t)gch * 2048 <= n) gch <<= 1;
    const uint32_t gchunks = (uint32_t)(((size_t)n + gch - 1) / gch);
    const uint32_t gain_blocks = std::min<uint32_t>(gchunks, 2048u);  // about one round of the scan
    // capacity of one proposal list: the vertices of its chunks
    const uint32_t slot_cap = chunk_slot_cap(gchunks) * gch;
    const uint32_t hub_blocks = dc[3] ? grid_for((dc[3] + S - 1) / S, 1, 256) : 0u;
    // hub gains: accumulators for every hub of the level (a sub-round lists
    // at most all of them), cleared once here and then by each pick
    int64_t *hacc = nullptr;
    unsigned long long *hU = nullptr;
    uint32_t *hcb = nullptr;
    const size_t hub_bytes = (size_t)dc[3] * ((64 * KW + 2) * 8 + 8 * KW + 4) + 3 * 256;
    if (dc[3] && A.remaining() >= hub_bytes) {  // else one workgroup per hub (k_gains_hub)
        hacc = A.alloc<int64_t>((size_t)dc[3] * (64 * KW + 2));
        hU = A.alloc<unsigned long long>((size_t)dc[3] * KW);
        hcb = A.alloc<uint32_t>((size_t)dc[3] + 1);
        fill<int64_t>(hacc, (size_t)dc[3] * (64 * KW + 2), 0, st);
        fill<unsigned long long>(hU, (size_t)dc[3] * KW, 0ull, st);
    }
    uint32_t *nhub = B.scal + 26;  // hub candidates of the sub-round (list in dlists)
    // grids of the per-sub-round kernels, sized by what one sub-round can hold
    // (about n / S proposals and movers); every kernel strides over its count
    const size_t per_sub = (size_t)n / S + 1;
    // (the kernels that read the proposal lists take a multiple of NSLOT)
    auto slot_grid = [](uint32_t g) { return (g + NSLOT - 1) / NSLOT * NSLOT; };
    const uint32_t fast_blocks = slot_grid(grid_for(per_sub, BLOCK, FILL_BLOCKS / 4));
    // gains of the listed candidates: one round of resident workgroups (six
    // per CU at 80 registers), so that every candidate's chain of dependent
    // gathers is in flight at once instead of in successive rounds
    const uint32_t list_blocks = slot_grid(6 * 256);
    // Small levels without hub vertices: the candidate lists of every
    // sub-round, built here once (k_lp_pre) in the space of k_gain_scan's
    // lists when they fit there, else from the workspace if it has room
    uint32_t *pre_lists = nullptr, *pre_off = nullptr;
    const uint32_t Rlp = std::min<uint32_t>(prm.lp_rounds, LP_MAX_ROUNDS);
    if (n && n < LP_PRE_N && !dc[3] && (uint64_t)Rlp * S <= LP_PRE_RS) {
        const size_t nent = (size_t)Rlp * S * 3 * NSLOT;
        auto words = [](size_t c) { return ((c * 4 + 255) & ~(size_t)255) / 4; };  // as the arena rounds
        const size_t need = words((size_t)Rlp * n) + words(nent + 1) + 2 * words(nent);
        uint32_t *base = nullptr;
        if (need <= 3 * ((size_t)n + (size_t)(3 * NSLOT) * GAIN_CH)) base = B.cl;
        else if (A.remaining() >= need * 4) base = A.alloc<uint32_t>(need);
        if (base) {
            pre_lists = base;
            pre_off = base + words((size_t)Rlp * n);
            uint32_t *cnt = pre_off + words(nent + 1), *cur = cnt + words(nent);
            fill<uint32_t>(cnt, nent, 0u, st);
            const uint32_t pb = std::min<uint32_t>(gchunks, FILL_BLOCKS);
            k_lp_pre<<<pb, BLOCK, 0, st>>>(h.inc_off, n, mseed, level, Rlp, S, gch, gchunks, cnt, nullptr, nullptr);
            HGP_LAUNCH_CHECK();
            k_lp_pre_scan<<<1, BLOCK, 0, st>>>(cnt, (uint32_t)nent, pre_off, cur);
            HGP_LAUNCH_CHECK();
            k_lp_pre<<<pb, BLOCK, 0, st>>>(h.inc_off, n, mseed, level, Rlp, S, gch, gchunks, nullptr, cur,
                                           pre_lists);
            HGP_LAUNCH_CHECK();
        }
    }
    // lanes per mover by the level's average degree (a lane per incident net)
    const uint64_t avg_deg = n ? ((uint64_t)h.p + n - 1) / n : 1;
    const uint32_t upd_g = avg_deg <= 8 ? 8u : (avg_deg <= 24 ? 16u : 64u);
    const uint32_t upd_blocks = slot_grid(grid_for(per_sub, BLOCK / upd_g, FILL_BLOCKS / 2));
    const uint32_t long_blocks = grid_for((size_t)m + 1, 64 * (BLOCK / WAVE), FILL_BLOCKS / 4);

    const int kb = bits_for(k - 1), ub = bits_for(n ? n - 1 : 0);
    // abort word: 1 + the sub-round whose selection handed a pair to the
    // device-wide path (0: none); later kernels of the round skip their work
    uint32_t *abort = B.scal + 15;
    // all per-sub-round state started at zero (afterwards the kernels of each
    // sub-round clear it for the next: the gains kernel what only later
    // kernels use, the update kernel the rest)
    const uint32_t seg_cap = pair_seg_cap(n);
    // proposal-list lengths of sub-round `stamp` (stamps are consecutive)
    auto pcnt_of = [&](uint32_t stamp) { return B.pcnt + (stamp & 1u) * NSLOT * SPREAD_U32; };
    const uint32_t pair_blocks = std::min<uint32_t>(k * (k - 1) / 2, 256u);
    uint32_t *nsp = B.scal + 25;  // over-budget pairs of the sub-round (list in spairs)

    // Device-wide selection of the pairs that sub-round (r, s) handed over
    // (more than PAIR_MAX proposals in one pair).  The counts are read back
    // here (the host has synchronised).
    auto slow_path = [&](uint32_t stamp) {
        // proposals of the flagged pairs
        uint32_t ns = 0;
        HGP_CHECK_HIP(hipMemsetAsync(nslow, 0, sizeof(uint32_t), st));
        k_collect_slow<<<fast_blocks, BLOCK, 0, st>>>(B.plist, pcnt_of(stamp), slot_cap, part, B.prop_t, k,
                                                      B.slowpair, B.slow, nslow);
        HGP_LAUNCH_CHECK();
        read_back(&ns, nslow, sizeof(uint32_t), st, false);
        HGP_CHECK_HIP(hipMemsetAsync(B.slowpair, 0, sizeof(uint32_t) * k * k, st));
        uint32_t G = 0;  // largest gain of the handed-over proposals
        if (ns) {
            HGP_CHECK_HIP(hipMemsetAsync(gmax, 0, sizeof(uint32_t), st));
            k_gain_max<<<grid_for(ns, BLOCK, 64), BLOCK, 0, st>>>(B.slow, ns, B.prop_g, gmax);
            HGP_LAUNCH_CHECK();
            read_back(&G, gmax, sizeof(uint32_t), st, false);
        }
        const int gb = bits_for(G);
        KeyLayout L;
        L.kmask = (1u << kb) - 1u;
        L.G = G;
        const bool fits = 2 * kb + gb + ub <= 64;
        const uint32_t *pl = B.slow;
        uint64_t *kk = B.keys;
        uint32_t *vv = B.vals;
        if (ns) {
            if (fits) {
                L.with_u = true;
                L.sh_u = 0; L.sh_g = ub; L.sh_t = ub + gb; L.sh_s = ub + gb + kb;
                k_lp_keys<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(pl, ns, part, B.prop_t, B.prop_g, L, kk,
                                                                             vv, false);
                HGP_LAUNCH_CHECK();
                radix_sort_pairs<uint64_t>(A, &kk, &vv, B.keys_alt, B.vals_alt, ns, 0, 2 * kb + gb + ub, st);
            } else {
                L.with_u = false;
                L.sh_u = 0; L.sh_g = 0; L.sh_t = gb; L.sh_s = gb + kb;
                k_u_only_keys<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(pl, ns, kk, vv);
                HGP_LAUNCH_CHECK();
                radix_sort_pairs<uint64_t>(A, &kk, &vv, B.keys_alt, B.vals_alt, ns, 0, ub, st);
                k_lp_keys<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(pl, ns, part, B.prop_t, B.prop_g, L, kk,
                                                                             vv, true);
                HGP_LAUNCH_CHECK();
                uint64_t *ka = (kk == B.keys) ? B.keys_alt : B.keys;
                uint32_t *va = (vv == B.vals) ? B.vals_alt : B.vals;
                radix_sort_pairs<uint64_t>(A, &kk, &vv, ka, va, ns, 0, 2 * kb + gb, st);
            }
            scan_apply<uint64_t>(A, ns, SortedWeight{vv, h.vwgt}, StoreIncl{B.incl}, (uint64_t *)nullptr, st);
            HGP_CHECK_HIP(hipMemsetAsync(B.seg_start, 0, sizeof(uint32_t) * k * k, st));
            HGP_CHECK_HIP(hipMemsetAsync(B.seg_end, 0, sizeof(uint32_t) * k * k, st));
            HGP_CHECK_HIP(hipMemsetAsync(B.best, 0, sizeof(unsigned long long) * k * k, st));
            k_pair_bounds<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(kk, ns, L, k, B.seg_start, B.seg_end);
            HGP_LAUNCH_CHECK();
            k_lp_select<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(kk, ns, L, k, B.seg_start, B.seg_end,
                                                                           B.incl, B.bw, lmax, B.best);
            HGP_LAUNCH_CHECK();
            k_lp_apply<<<grid_for(ns, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(kk, vv, ns, L, k, B.seg_start, B.best,
                                                                          h.vwgt, part, B.bw);
            HGP_LAUNCH_CHECK();
        }
        k_add_dbw<<<1, 256, 0, st>>>(B.bw, B.dbw_g, k);
        HGP_LAUNCH_CHECK();
    };
    // Update of the nets touched by the sub-round's moves.
    auto ctl_of = [&](uint32_t stamp) {
        const uint32_t r = (stamp - 1) / S;
        return LpCtl{abort, r ? B.rmoves + r - 1 : nullptr, stamp};
    };
    auto update = [&](uint32_t stamp) {
        const LpCtl ctl = ctl_of(stamp);
        uint32_t *moved = B.rmoves + (stamp - 1) / S;
        if (accounting(KID_LP_UPDATE)) {
            Timing &T = timing();
            ++T.stamp;
            static_assert((FILL_BLOCKS / 4) % NSLOT == 0, "the proposal lists need a multiple of NSLOT");
            k_account_update<KW><<<FILL_BLOCKS / 4, BLOCK, 0, st>>>(h.pin_off, h.inc_off, h.inc, B.plist,
                                                                    pcnt_of(stamp), slot_cap, part, B.prop_t,
                                                                    T.marks, T.stamp,
                                                                    (unsigned long long *)T.acc_dev + KID_LP_UPDATE,
                                                                    ctl);
            HGP_LAUNCH_CHECK();
        }
        {
            TimedLaunch tl(KID_LP_UPDATE, st);
            const NextSub zn{B.scal, B.pw, B.pc, B.pcur, B.ccnt, k * k, k, B.bw, B.dbw_g, pcnt_of(stamp + 1)};
            auto launch = [&](auto kern, uint32_t blocks) {
                kern<<<blocks, BLOCK, 0, st>>>(h.pin_off, h.pins, h.inc_off, h.inc, B.plist, pcnt_of(stamp), slot_cap,
                                               B.prop_t, part, (NetRec<KW> *)B.nr, B.tstamp, stamp, B.f, B.longl,
                                               nlong, moved, B.bcnt, B.heavy, nheavy, zn, ctl, gupd);
            };
            if (upd_g == 8) launch(k_lp_update_movers<KW, 8>, upd_blocks);
            else if (upd_g == 16) launch(k_lp_update_movers<KW, 16>, upd_blocks);
            else launch(k_lp_update_movers<KW, 64>, upd_blocks);
            HGP_LAUNCH_CHECK();
        }
        if (dc[3]) {  // the level has nodes of more than HUB_DEG nets
            k_heavy_chunks<<<1, HEAVY_SCAN, 0, st>>>(h.inc_off, B.heavy, nheavy, B.hcbase);
            HGP_LAUNCH_CHECK();
            k_lp_update_heavy<KW><<<FILL_BLOCKS / 2, BLOCK, 0, st>>>(h.pin_off, h.pins, h.inc_off, h.inc, B.heavy,
                                                                   nheavy, B.hcbase, part, (NetRec<KW> *)B.nr,
                                                                   B.tstamp, stamp, B.f, B.longl, nlong, B.bcnt,
                                                                   ctl, gupd);
            HGP_LAUNCH_CHECK();
        }
        if (long_nets) {
            k_conn_long<KW><<<long_blocks, BLOCK, 0, st>>>(h.pin_off, h.pins, B.longl, nlong, h.nwgt, part,
                                                           (NetRec<KW> *)B.nr, B.f, true, B.bcnt, ctl);
            HGP_LAUNCH_CHECK();
        }
    };
    // One sub-round, entirely on the device (no host round trip).
    auto subround = [&](uint32_t r, uint32_t s) {
        const uint32_t stamp = 1 + r * S + s;
        const LpCtl ctl = ctl_of(stamp);
        GainArgs<KW> ga{h.inc_off, h.inc, h.vwgt, (const NetRec<KW> *)B.nr, part, B.bw, B.bcnt, lmax, mseed,
                              level, r, s, S, n, B.prop_t, B.prop_g, B.plist, pcnt_of(stamp), gch, slot_cap,
                              B.pw, B.pc, k, ctl};
        ga.adj = adj;
        ga.adjw = adjw;
        if (accounting(KID_GAINS)) {
            Timing &T = timing();
            ++T.stamp;
            k_account_gains<KW><<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(
                ga, T.marks, T.stamp, (unsigned long long *)T.acc_dev + KID_GAINS);
            HGP_LAUNCH_CHECK();
        }
        if (n && pre_lists) {
            const uint32_t *po = pre_off + (size_t)(r * S + s) * 3 * NSLOT;
            TimedLaunch tl(KID_GAINS, st);
            if (adj) k_gains<KW, true><<<list_blocks, BLOCK, 0, st>>>(ga, pre_lists, nullptr, po, B.scal);
            else k_gains<KW, false><<<list_blocks, BLOCK, 0, st>>>(ga, pre_lists, nullptr, po, B.scal);
            HGP_LAUNCH_CHECK();
        } else if (n) {
            k_gain_scan<KW><<<gain_blocks, BLOCK, 0, st>>>(ga, gch, gchunks, B.cl, B.ccnt, B.dlists, nhub, B.scal);
            HGP_LAUNCH_CHECK();
            TimedLaunch tl(KID_GAINS, st);
            if (adj) k_gains<KW, true><<<list_blocks, BLOCK, 0, st>>>(ga, B.cl, B.ccnt, nullptr, nullptr);
            else k_gains<KW, false><<<list_blocks, BLOCK, 0, st>>>(ga, B.cl, B.ccnt, nullptr, nullptr);
            HGP_LAUNCH_CHECK();
        }
        if (hub_blocks && !hacc) {
            if (adj) k_gains_hub<KW, true><<<hub_blocks, HUB_THREADS, 0, st>>>(ga, B.dlists, nhub);
            else k_gains_hub<KW, false><<<hub_blocks, HUB_THREADS, 0, st>>>(ga, B.dlists, nhub);
            HGP_LAUNCH_CHECK();
        } else if (hub_blocks) {
            k_heavy_chunks<<<1, HEAVY_SCAN, 0, st>>>(h.inc_off, B.dlists, nhub, hcb, HUB_GCH);
            HGP_LAUNCH_CHECK();
            if (adj)
                k_gains_hub_part<KW, true><<<FILL_BLOCKS / 2, HUB_THREADS, 0, st>>>(ga, B.dlists, nhub, hcb, hacc, hU);
            else
                k_gains_hub_part<KW, false><<<FILL_BLOCKS / 2, HUB_THREADS, 0, st>>>(ga, B.dlists, nhub, hcb, hacc, hU);
            HGP_LAUNCH_CHECK();
            k_gains_hub_pick<KW><<<hub_blocks, BLOCK, 0, st>>>(ga, B.dlists, nhub, hacc, hU);
            HGP_LAUNCH_CHECK();
        }
        {  // pairs whose whole move sets are feasible: applied directly
            TimedLaunch tl(KID_LP_FAST, st);
            k_lp_fast<<<fast_blocks, BLOCK, 0, st>>>(B.plist, pcnt_of(stamp), slot_cap, B.prop_t, B.pw, k, h.vwgt,
                                                     part, B.bw, lmax, B.dbw_g, B.pcur, B.seg, seg_cap, B.spairs,
                                                     nsp, ctl);
            HGP_LAUNCH_CHECK();
        }
        {  // the other pairs: sorted two-pointer walk, a workgroup per pair
            TimedLaunch tl(KID_LP_PAIRS, st);
            k_lp_pairs<<<pair_blocks, PAIR_THREADS, 0, st>>>(B.spairs, nsp, B.pc, B.seg, seg_cap, k, B.prop_g,
                                                             h.vwgt, part, B.bw, lmax, B.dbw_g, B.slowpair, ctl);
            HGP_LAUNCH_CHECK();
        }
        update(stamp);
    };

    // Rounds are queued LP_ROUND_BATCH at a time with one read-back per
    // batch: a round after one without moves does nothing on the device, and
    // a sub-round handed to the device-wide path stops every later one until
    // the host has finished it; the rest is then queued again.
    // After a hand-over the level queues one round at a time (levels that
    // need the device-wide path tend to need it again: a batch would be
    // queued, skipped and queued again).
    const uint32_t R = std::min<uint32_t>(prm.lp_rounds, LP_MAX_ROUNDS);
    uint32_t r0 = 0, s0 = 0;  // next sub-round to queue
    uint32_t batch = LP_ROUND_BATCH;
    uint32_t rounds_run = 0;
    while (r0 < R) {
        const uint32_t r1 = std::min<uint32_t>(R, r0 + batch);
        for (uint32_t r = r0; r < r1; ++r)
            for (uint32_t s = (r == r0 ? s0 : 0); s < S; ++s) subround(r, s);
        uint32_t hv[1 + LP_ROUND_BATCH];
        read_back({{&hv[0], abort, sizeof(uint32_t)}, {&hv[1], B.rmoves + r0, sizeof(uint32_t) * (r1 - r0)}}, st,
                  false);
        if (hv[0]) {
            // sub-round hv[0] handed pairs to the device-wide path: finish it
            // there, then queue the sub-rounds after it again
            const uint32_t stamp = hv[0];
            HGP_CHECK_HIP(hipMemsetAsync(abort, 0, sizeof(uint32_t), st));
            slow_path(stamp);
            update(stamp);
            r0 = (stamp - 1) / S;
            s0 = (stamp - 1) % S + 1;
            rounds_run = r0 + 1;
            batch = 1;
            if (s0 == S) {
                // the hand-over finished its round: a round without moves
                // ends LP here as well
                uint32_t mv = 0;
                read_back(&mv, B.rmoves + r0, sizeof(uint32_t), st, false);
                if (mv == 0) break;
                ++r0;
                s0 = 0;
            }
            continue;
        }
        // a round without moves ends LP (the rounds after it did nothing)
        bool stop = false;
        for (uint32_t r = r0; r < r1 && !stop; ++r) {
            rounds_run = r + 1;
            stop = hv[1 + (r - r0)] == 0;
        }
        if (stop) break;
        r0 = r1;
        s0 = 0;
    }
    if (rounds_out) *rounds_out = rounds_run;
    // the last sub-round's block-weight changes
    k_add_dbw<<<1, 256, 0, st>>>(B.bw, B.dbw_g, k);
    HGP_LAUNCH_CHECK();
    if (obj) {
        k_objective_total<<<1, WAVE, 0, st>>>(B.f, obj);
        HGP_LAUNCH_CHECK();
    }
    if (bw_out) HGP_CHECK_HIP(hipMemcpyAsync(bw_out, B.bw, sizeof(int64_t) * k, hipMemcpyDeviceToDevice, st));
    stream_sync(st);
    A.release(mk);
}

void refine_lp(const hgp_hg &h, const hgp_params &prm, uint32_t level, uint32_t *part, int64_t *obj, int64_t *bw,
               Arena &A, hipStream_t st, int64_t W_known, uint32_t *rounds_out, const int64_t *side_limits) {
    switch ((prm.k + 63) / 64) {
        case 1: refine_t<1>(h, prm, level, part, obj, bw, A, st, W_known, rounds_out, side_limits); break;
        case 2: refine_t<2>(h, prm, level, part, obj, bw, A, st, W_known, rounds_out, side_limits); break;
        case 3: refine_t<3>(h, prm, level, part, obj, bw, A, st, W_known, rounds_out, side_limits); break;
        default: refine_t<4>(h, prm, level, part, obj, bw, A, st, W_known, rounds_out, side_limits); break;
    }
}

}  // namespace hgp
