// Greedy initial partition of the coarsest level (a simple deterministic
// method; the paper's portfolio of Sec. 5 is not part of this path) and the
// projection step of uncoarsening (Sec. 3).
//
// Order: breadth-first from the smallest unvisited vertex, neighbours taken
// in ascending incident-net order and, inside a net, ascending pin order.
// The order is built one BFS layer at a time with device-wide kernels: the
// (frontier vertex, incident net) pairs of a layer are numbered by a scan
// of the frontier degrees; every occurrence of an unvisited vertex gets the
// key (frontier position, offset in that vertex's expansion), so a vertex
// joins the next layer at its smallest key; winners are counted per pair and
// laid out in pair order by a second scan, which is exactly key order.
// Vertices without incident nets can never be reached and are appended in
// ID order whenever the search passes them.
// Fill: block b covers positions [S_b, S_{b+1}) of the order, where
// S_{b+1} = 1 + first i >= S_b with weight(S_b..i) >= ceil(c(V)/k); the S_b
// are found by pointer doubling over next(s), the last block takes the rest.
#include "prims.h"
#include "kernels.h"

namespace hgp {

// expansion offset of every incidence entry: sum of the sizes of the
// earlier nets of the same vertex
__global__ __launch_bounds__(BLOCK) void k_exoff(const uint32_t *pin_off, const uint32_t *inc_off,
                                                 const uint32_t *inc, uint32_t n, uint32_t *exoff) {
    // exclusive prefix of the sizes of each vertex's nets; a vertex of more
    // than 128 nets is scanned by its whole wave, 64 entries at a time (a
    // wave takes its heavy vertices one after another, so the threshold is
    // above the degrees of coarse levels, which run to a few dozen)
    for (uint32_t v0 = blockIdx.x * BLOCK; v0 < n; v0 += gridDim.x * BLOCK) {
        const uint32_t v = v0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (v < n) { j0 = inc_off[v]; j1 = inc_off[v + 1]; }
        const bool heavy = j1 - j0 > 128;
        if (!heavy) {  // eight nets at a time: their IDs, then their sizes, then the prefix
            uint32_t acc = 0;
            for (uint32_t j = j0; j < j1; j += 8) {
                uint32_t ev[8], sz[8];
#pragma unroll
                for (uint32_t c = 0; c < 8; ++c) ev[c] = j + c < j1 ? inc[j + c] : NONE;
#pragma unroll
                for (uint32_t c = 0; c < 8; ++c) sz[c] = ev[c] != NONE ? pin_off[ev[c] + 1] - pin_off[ev[c]] : 0u;
#pragma unroll
                for (uint32_t c = 0; c < 8; ++c) {
                    if (j + c < j1) exoff[j + c] = acc;
                    acc += sz[c];
                }
            }
        }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int h = __ffsll((long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t hj0 = __shfl(j0, h, 64), hj1 = __shfl(j1, h, 64);
            uint32_t carry = 0;
            for (uint32_t b = hj0; b < hj1; b += WAVE) {
                const uint32_t j = b + __lane_id();
                uint32_t x = 0;
                if (j < hj1) {
                    const uint32_t e = inc[j];
                    x = pin_off[e + 1] - pin_off[e];
                }
                uint32_t incl = x;  // inclusive wave scan
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o, 64);
                    if ((int)__lane_id() >= o) incl += y;
                }
                if (j < hj1) exoff[j] = carry + incl - x;
                carry += __shfl(incl, 63, 64);
            }
        }
    }
}

// smallest unvisited vertex with incident nets in [from, n) -> *out (preset n)
__global__ void k_find_start(const uint32_t *inc_off, const uint32_t *visited, uint32_t from, uint32_t n,
                             uint32_t *out) {
    uint32_t best = n;
    for (uint32_t v = from + blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (!visited[v] && inc_off[v + 1] > inc_off[v]) { best = v; break; }  // ascending per thread
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(best, o, 64);
        best = y < best ? y : best;
    }
    if (__lane_id() == 0 && best < n) atomicMin(out, best);  // one atomic per wave
}

struct Unvisited {
    const uint32_t *visited;
    uint32_t from;
    __device__ uint32_t operator()(size_t i) const { return visited[from + i] ? 0u : 1u; }
};
struct AppendOrder {
    const uint32_t *visited;
    uint32_t *order, *vis_w;
    uint32_t from, pos;
    __device__ void operator()(size_t i, uint32_t excl, uint32_t v) const {
        if (v) order[pos + excl] = from + (uint32_t)i;
    }
};

// State of a BFS layer in device memory (two copies, by layer parity): the
// frontier order[fs, fs + F), the next free order position, and the layer's
// expansion size T and winner count W once known.
enum BfsWord { BFS_FS = 0, BFS_POS = 1, BFS_F = 2, BFS_T = 3, BFS_W = 4, BFS_WORDS = 8 };

__global__ void k_mark_range(const uint32_t *order, uint32_t a, uint32_t b, uint32_t *visited,
                             unsigned long long *key) {
    for (uint32_t i = a + blockIdx.x * blockDim.x + threadIdx.x; i < b; i += gridDim.x * blockDim.x) {
        uint32_t w = order[i];
        visited[w] = 1;
        key[w] = ~0ull;
    }
}

// The start vertex opens a BFS: order[pos] = s, the first layer state.
// One device word from a host value (a kernel argument, not a copy from
// pageable host memory).
__global__ void k_put_u32(uint32_t *p, uint32_t v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

__global__ void k_put_start(uint32_t *order, uint32_t pos, const uint32_t *start, uint32_t *visited, uint32_t *bst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t s = *start;
        order[pos] = s;
        visited[s] = 1;
        bst[BFS_FS] = pos;
        bst[BFS_POS] = pos + 1;
        bst[BFS_F] = 1;
    }
}

// Layer winners [pos, pos + W) become visited; the next layer's state (the
// other copy) has them as its frontier.
__global__ void k_bfs_mark(const uint32_t *order, const uint32_t *cur, uint32_t *nxt, uint32_t *visited,
                           unsigned long long *key, uint32_t *base) {
    const uint32_t a = cur[BFS_POS], W = cur[BFS_W];
    for (uint32_t i = a + blockIdx.x * blockDim.x + threadIdx.x; i < a + W; i += gridDim.x * blockDim.x) {
        uint32_t w = order[i];
        visited[w] = 1;
        key[w] = ~0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        nxt[BFS_FS] = a;
        nxt[BFS_POS] = a + W;
        nxt[BFS_F] = W;
        if (base) *base += cur[BFS_T];  // the next layer's pairs number on from here
    }
}

struct FrontierDeg {
    const uint32_t *order, *inc_off;
    const uint32_t *fs;
    __device__ uint32_t operator()(size_t i) const {
        uint32_t v = order[*fs + i];
        return inc_off[v + 1] - inc_off[v];
    }
};

// flat pair t -> (frontier index fi, incidence index jj)
__device__ inline void pair_of(const uint32_t *D, uint32_t F, uint32_t t, const uint32_t *order, uint32_t fs,
                               const uint32_t *inc_off, uint32_t &fi, uint32_t &jj) {
    uint32_t lo = 0, hi = F - 1;  // largest fi with D[fi] <= t
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (D[mid] <= t) lo = mid; else hi = mid - 1;
    }
    fi = lo;
    jj = inc_off[order[fs + fi]] + (t - D[fi]);
}

// Expanding each net once (when nets are large against the pins): the
// first pair of the layer that reaches a net is the only one to expand it,
// because all of the net's pins join in that layer and its later pairs add
// nothing.  netT[e] holds the first pair number (pair numbers grow over the
// layers: *base + t), so a net expanded in an earlier layer is below *base.
// The expansion index of a pin through its net's first pair is the smallest
// through any pair of the net, so the keys and the order do not change.
__global__ void k_bfs_first(const uint32_t *D, const uint32_t *bst, const uint32_t *order, const uint32_t *inc_off,
                            const uint32_t *inc, const uint32_t *base, uint32_t *netT) {
    const uint32_t F = bst[BFS_F], T = bst[BFS_T], fs = bst[BFS_FS], b0 = *base;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
        uint32_t fi, jj;
        pair_of(D, F, t, order, fs, inc_off, fi, jj);
        const uint32_t e = inc[jj];
        if (netT[e] >= b0) atomicMin(&netT[e], b0 + t);
    }
}

// Pair t expands its net: always, or (netT set) only as the net's first pair.
__device__ inline bool expands(const uint32_t *netT, const uint32_t *base, uint32_t e, uint32_t t) {
    return !netT || netT[e] == *base + t;
}

__global__ void k_bfs_keys(const uint32_t *D, const uint32_t *bst, const uint32_t *order, const uint32_t *inc_off,
                           const uint32_t *inc, const uint32_t *pin_off, const uint32_t *pins,
                           const uint32_t *exoff, const uint32_t *visited, unsigned long long *key,
                           const uint32_t *netT, const uint32_t *base) {
    const uint32_t F = bst[BFS_F], T = bst[BFS_T], fs = bst[BFS_FS];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
        uint32_t fi, jj;
        pair_of(D, F, t, order, fs, inc_off, fi, jj);
        uint32_t e = inc[jj];
        if (!expands(netT, base, e, t)) continue;
        uint64_t base = ((uint64_t)fi << 32) | exoff[jj];
        const uint32_t b = pin_off[e], b1 = pin_off[e + 1];
        for (uint32_t q0 = b; q0 < b1; q0 += 8) {  // eight pins at a time: pins, then their flags
            uint32_t w[8], vis[8];
#pragma unroll
            for (uint32_t c = 0; c < 8; ++c) w[c] = q0 + c < b1 ? pins[q0 + c] : NONE;
#pragma unroll
            for (uint32_t c = 0; c < 8; ++c) vis[c] = w[c] != NONE ? visited[w[c]] : 1u;
#pragma unroll
            for (uint32_t c = 0; c < 8; ++c)
                if (!vis[c]) atomicMin(&key[w[c]], (unsigned long long)(base + (q0 + c - b)));
        }
    }
}

// winners of pair t: count (write=false) or append in key order (write=true)
__global__ void k_bfs_winners(const uint32_t *D, const uint32_t *bst, const uint32_t *order,
                              const uint32_t *inc_off, const uint32_t *inc, const uint32_t *pin_off,
                              const uint32_t *pins, const uint32_t *exoff, const uint32_t *visited,
                              const unsigned long long *key, uint32_t *cnt, uint32_t *order_out, bool write,
                              const uint32_t *netT, const uint32_t *base) {
    const uint32_t F = bst[BFS_F], T = bst[BFS_T], fs = bst[BFS_FS], pos = bst[BFS_POS];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
        uint32_t fi, jj;
        pair_of(D, F, t, order, fs, inc_off, fi, jj);
        uint32_t e = inc[jj];
        if (!expands(netT, base, e, t)) {
            if (!write) cnt[t] = 0;
            continue;
        }
        uint64_t base = ((uint64_t)fi << 32) | exoff[jj];
        const uint32_t b = pin_off[e], b1 = pin_off[e + 1];
        uint32_t c = 0, wp = write ? pos + cnt[t] : 0;
        for (uint32_t q0 = b; q0 < b1; q0 += 8) {  // eight pins at a time, decided in pin order
            uint32_t w[8], vis[8];
            unsigned long long kw[8];
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) w[i] = q0 + i < b1 ? pins[q0 + i] : NONE;
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) {
                vis[i] = w[i] != NONE ? visited[w[i]] : 1u;
                kw[i] = w[i] != NONE ? key[w[i]] : 0ull;
            }
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) {
                if (!vis[i] && kw[i] == base + (q0 + i - b)) {
                    if (write) order_out[wp + c] = w[i];
                    ++c;
                }
            }
        }
        if (!write) cnt[t] = c;
    }
}

struct OrderWeight {
    const uint32_t *order;
    const int32_t *vwgt;
    __device__ uint64_t operator()(size_t i) const { return (uint64_t)(uint32_t)vwgt[order[i]]; }
};
struct StoreInclP {
    uint64_t *P;
    __device__ void operator()(size_t i, uint64_t excl, uint64_t v) const { P[i] = excl + v; }
};

// J0[s] = next(s) for s in [0, n]
__global__ void k_next(const uint64_t *P, uint32_t n, uint64_t T, uint32_t *J0) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s <= n; s += gridDim.x * blockDim.x) {
        if (s >= n) { J0[s] = n; continue; }
        uint64_t target = (s == 0 ? 0 : P[s - 1]) + T;
        uint32_t lo = s, hi = n;  // first i in [s, n) with P[i] >= target, or n
        while (lo < hi) {
            uint32_t mid = lo + ((hi - lo) >> 1);
            if (P[mid] >= target) hi = mid; else lo = mid + 1;
        }
        J0[s] = lo < n ? lo + 1 : n;
    }
}

__global__ void k_jump(const uint32_t *Jin, uint32_t n, uint32_t *Jout) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s <= n; s += gridDim.x * blockDim.x)
        Jout[s] = Jin[Jin[s]];
}

__global__ void k_starts(const uint32_t *J, uint32_t n, uint32_t k, int levels, uint32_t *S) {
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < k; b += gridDim.x * blockDim.x) {
        uint32_t s = 0;
        for (int l = 0; l < levels; ++l)
            if ((b >> l) & 1u) s = J[(size_t)l * (n + 1) + s];
        S[b] = s;
    }
}

__global__ void k_assign(const uint32_t *order, uint32_t n, const uint32_t *S, uint32_t k, uint32_t *part) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = k - 1;  // largest b with S[b] <= i (S[0] = 0)
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (S[mid] <= i) lo = mid; else hi = mid - 1;
        }
        part[order[i]] = lo;
    }
}

__global__ void k_project(uint32_t n, const uint32_t *cid, const uint32_t *cpart, uint32_t *part) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        part[v] = cpart[cid[v]];
}

// ---------------------------------------------------------------------------
// Small coarsest levels: the whole order and fill in one workgroup (no host
// round trip per layer).  The order is the same: within a layer the
// expansion (frontier vertex, incident net, pin) is flattened to one index x
// in lexicographic order, which is the key order of the device-wide path, so
// a vertex joins the next layer at its smallest x and the winners are laid
// out in x order.  Only the first pair that reaches a net expands it (its
// pins all join in that layer), so a BFS expands every net once: about one
// workgroup step per IPS_THREADS pins and incidences.  Used when the sum over
// nets of |e|^2 is small.
// ---------------------------------------------------------------------------
constexpr int IPS_THREADS = 1024;
constexpr uint32_t IPS_MAX_N = 1u << 16;
constexpr uint32_t IPS_MAX_P = 1u << 20;
constexpr uint64_t IPS_MAX_SQ = 1ull << 18;  // sum over nets of |e|^2

// sum over nets of |e|^2
__global__ void k_sq_sizes(const uint32_t *pin_off, uint32_t m, unsigned long long *out) {
    unsigned long long acc = 0;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
        const unsigned long long z = pin_off[e + 1] - pin_off[e];
        acc += z * z;
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0 && acc) atomicAdd(out, acc);
}

__device__ inline uint32_t ips_min(uint32_t v, uint32_t *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(v, o, 64);
        v = y < v ? y : v;
    }
    __syncthreads();
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    uint32_t r = red[0];
    for (int i = 1; i < IPS_THREADS / WAVE; ++i) r = red[i] < r ? red[i] : r;
    __syncthreads();  // red is reused by the caller
    return r;
}

// Owner lookups over an exclusive prefix A[0..len) of positive sizes
// (A[0] = 0): the owner of position x is the largest i with A[i] <= x.  A
// window of IPS_THREADS consecutive positions starting at c0 is covered by
// at most IPS_THREADS + 1 segments starting at the owner of c0 (`cur`), so
// those starts are staged in LDS and every lookup is an LDS search.
template <class T>
__device__ inline void ips_stage(const T *A, uint32_t len, uint32_t cur, T *win) {
    for (uint32_t j = threadIdx.x; j <= (uint32_t)IPS_THREADS; j += IPS_THREADS)
        win[j] = cur + j < len ? A[cur + j] : ~(T)0;
    __syncthreads();
}
template <class T>
__device__ inline uint32_t ips_owner(const T *win, uint32_t cur, T x) {
    uint32_t lo = 0, hi = IPS_THREADS;  // largest j with win[j] <= x (win[0] <= x)
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (win[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return cur + lo;
}

__global__ __launch_bounds__(IPS_THREADS) void k_ip_small(const uint32_t *pin_off, const uint32_t *pins,
                                                          const uint32_t *inc_off, const uint32_t *inc,
                                                          const int32_t *vwgt, uint32_t n, uint32_t k, uint64_t T,
                                                          unsigned long long *key, uint32_t *D, uint32_t *pe,
                                                          uint64_t *E, uint32_t *order, uint64_t *P, uint32_t *S,
                                                          uint32_t *part, uint32_t *netT, uint32_t m) {
    __shared__ uint32_t red[IPS_THREADS / WAVE];
    __shared__ uint64_t red64[IPS_THREADS / WAVE];
    __shared__ uint32_t vis[IPS_MAX_N / 32];  // visited bitmap
    __shared__ uint64_t win[IPS_THREADS + 1];
    __shared__ uint32_t win32[IPS_THREADS + 1];
    const uint32_t tid = threadIdx.x;
    auto visited = [&](uint32_t v) -> bool { return (vis[v >> 5] >> (v & 31)) & 1u; };
    auto visit = [&](uint32_t v) { atomicOr(&vis[v >> 5], 1u << (v & 31)); };
    for (uint32_t i = tid; i < (n + 31) / 32; i += IPS_THREADS) vis[i] = 0;
    for (uint32_t v = tid; v < n; v += IPS_THREADS) key[v] = ~0ull;
    for (uint32_t e = tid; e < m; e += IPS_THREADS) netT[e] = ~0u;  // first pair of every net: none yet
    __syncthreads();
    uint32_t pos = 0, next = 0;
    uint32_t base = 0;  // pairs of the earlier layers
    while (pos < n) {
        // smallest unvisited vertex with incident nets at or after `next`;
        // the unvisited vertices before it have no nets and join in ID order
        uint32_t s = n;
        for (uint32_t c0 = next; c0 < n; c0 += IPS_THREADS) {
            const uint32_t v = c0 + tid;
            const bool cand = v < n && !visited(v) && inc_off[v + 1] > inc_off[v];
            s = ips_min(cand ? v : n, red);
            if (s < n) break;
        }
        for (uint32_t c0 = next; c0 < s; c0 += IPS_THREADS) {
            const uint32_t v = c0 + tid;
            const uint32_t un = (v < s && !visited(v)) ? 1u : 0u;
            uint32_t tot;
            const uint32_t incl = block_incl_scan_n<uint32_t, IPS_THREADS>(un, red, &tot);
            if (un) {
                order[pos + incl - 1] = v;
                visit(v);
            }
            pos += tot;
        }
        if (s >= n) break;
        if (tid == 0) { order[pos] = s; visit(s); }
        uint32_t fs = pos, fe = pos + 1;
        pos += 1;
        next = s + 1;
        __syncthreads();
        while (fs < fe) {
            const uint32_t F = fe - fs;
            // D: exclusive prefix of the frontier degrees (pairs of the layer)
            uint32_t Tn = 0;
            for (uint32_t c0 = 0; c0 < F; c0 += IPS_THREADS) {
                const uint32_t i = c0 + tid;
                uint32_t d = 0;
                if (i < F) {
                    const uint32_t v = order[fs + i];
                    d = inc_off[v + 1] - inc_off[v];
                }
                uint32_t tot;
                const uint32_t incl = block_incl_scan_n<uint32_t, IPS_THREADS>(d, red, &tot);
                if (i < F) D[i] = Tn + incl - d;
                Tn += tot;
            }
            __syncthreads();
            // A net's pins join at the first pair (frontier vertex, incident
            // net) that reaches it, and they are all visited in that layer:
            // so each net is expanded once, at its first pair (pair numbers
            // grow over the layers: base + t), and a vertex's smallest
            // expansion index over the expanded nets is its smallest over
            // every pair of the layer.
            uint32_t cur = 0;  // frontier index owning pair c0
            for (uint32_t c0 = 0; c0 < Tn; c0 += IPS_THREADS) {
                ips_stage<uint32_t>(D, F, cur, win32);
                const uint32_t t = c0 + tid;
                if (t < Tn) {
                    const uint32_t fi = ips_owner<uint32_t>(win32, cur, t);
                    const uint32_t e = inc[inc_off[order[fs + fi]] + (t - D[fi])];
                    pe[t] = e;
                    if (netT[e] >= base) atomicMin(&netT[e], base + t);
                }
                cur = ips_owner<uint32_t>(win32, cur, c0 + IPS_THREADS);
                __syncthreads();  // the window is restaged
            }
            __syncthreads();
            // the layer's expanded nets in pair order (compacted in place: a
            // chunk's reads precede its scans' barriers, its writes land
            // below the next chunk) with E = exclusive prefix of their sizes
            uint64_t X = 0;
            uint32_t Tx = 0;
            for (uint32_t c0 = 0; c0 < Tn; c0 += IPS_THREADS) {
                const uint32_t t = c0 + tid;
                uint32_t e = 0, first = 0;
                uint64_t sz = 0;
                if (t < Tn) {
                    e = pe[t];
                    first = netT[e] == base + t ? 1u : 0u;
                    sz = first ? pin_off[e + 1] - pin_off[e] : 0u;
                }
                uint32_t totf;
                const uint32_t incf = block_incl_scan_n<uint32_t, IPS_THREADS>(first, red, &totf);
                uint64_t tots;
                const uint64_t incs = block_incl_scan_n<uint64_t, IPS_THREADS>(sz, red64, &tots);
                if (first) {
                    pe[Tx + incf - 1] = e;
                    E[Tx + incf - 1] = X + incs - sz;
                }
                Tx += totf;
                X += tots;
            }
            __syncthreads();
            base += Tn;
            // keys: smallest expansion index per unvisited vertex
            cur = 0;
            for (uint64_t c0 = 0; c0 < X; c0 += IPS_THREADS) {
                ips_stage<uint64_t>(E, Tx, cur, win);
                const uint64_t x = c0 + tid;
                if (x < X) {
                    const uint32_t t = ips_owner<uint64_t>(win, cur, x);
                    const uint32_t e = pe[t];
                    const uint32_t w = pins[pin_off[e] + (uint32_t)(x - E[t])];
                    if (!visited(w)) atomicMin(&key[w], (unsigned long long)x);
                }
                cur = ips_owner<uint64_t>(win, cur, c0 + IPS_THREADS);
                __syncthreads();  // the window is restaged
            }
            // winners in expansion order
            uint32_t Wn = 0;
            cur = 0;
            for (uint64_t c0 = 0; c0 < X; c0 += IPS_THREADS) {
                ips_stage<uint64_t>(E, Tx, cur, win);
                const uint64_t x = c0 + tid;
                uint32_t w = 0, wn = 0;
                if (x < X) {
                    const uint32_t t = ips_owner<uint64_t>(win, cur, x);
                    const uint32_t e = pe[t];
                    w = pins[pin_off[e] + (uint32_t)(x - E[t])];
                    // the key is read back at L2, where the atomics were applied
                    wn = (!visited(w) && atomicOr(&key[w], 0ull) == x) ? 1u : 0u;
                }
                cur = ips_owner<uint64_t>(win, cur, c0 + IPS_THREADS);
                uint32_t tot;
                const uint32_t incl = block_incl_scan_n<uint32_t, IPS_THREADS>(wn, red, &tot);
                if (wn) order[pos + Wn + incl - 1] = w;
                Wn += tot;
            }
            __syncthreads();
            for (uint32_t i = pos + tid; i < pos + Wn; i += IPS_THREADS) {
                const uint32_t w = order[i];
                visit(w);
                atomicExch(&key[w], ~0ull);
            }
            __syncthreads();
            fs = pos;
            fe = pos + Wn;
            pos += Wn;
        }
    }
    __syncthreads();
    // fill: P = inclusive prefix of the weights in order
    uint64_t carry = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += IPS_THREADS) {
        const uint32_t i = c0 + tid;
        const uint64_t w = i < n ? (uint64_t)(uint32_t)vwgt[order[i]] : 0ull;
        uint64_t tot;
        const uint64_t incl = block_incl_scan_n<uint64_t, IPS_THREADS>(w, red64, &tot);
        if (i < n) P[i] = carry + incl;
        carry += tot;
    }
    __syncthreads();
    // block b starts at S_b; S_{b+1} = 1 + first i >= S_b whose prefix from
    // S_b reaches T (the last block takes the rest)
    if (tid == 0) {
        uint32_t sb = 0;
        S[0] = 0;
        for (uint32_t b = 1; b < k; ++b) {
            if (sb < n) {
                const uint64_t target = (sb == 0 ? 0ull : P[sb - 1]) + T;
                uint32_t lo = sb, hi = n;  // first i in [sb, n) with P[i] >= target, or n
                while (lo < hi) {
                    const uint32_t mid = lo + ((hi - lo) >> 1);
                    if (P[mid] >= target) hi = mid; else lo = mid + 1;
                }
                sb = lo < n ? lo + 1 : n;
            }
            S[b] = sb;
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += IPS_THREADS) {
        uint32_t lo = 0, hi = k - 1;  // largest b with S[b] <= i
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (S[mid] <= i) lo = mid; else hi = mid - 1;
        }
        part[order[i]] = lo;
    }
}

struct IpBufs {
    uint32_t *order, *visited, *J, *S, *exoff, *D, *cnt, *scal, *netT;
    uint32_t *bst;  // [2][BFS_WORDS] BFS layer states
    unsigned long long *key;
    uint64_t *P, *E;
};

static void plan(Arena &A, uint32_t n, uint32_t m, uint32_t p, uint32_t k, IpBufs &B) {
    B.netT = A.alloc<uint32_t>(m ? m : 1);
    B.order = A.alloc<uint32_t>(n);
    B.visited = A.alloc<uint32_t>(n);
    B.key = A.alloc<unsigned long long>(n);
    B.P = A.alloc<uint64_t>(n);
    B.J = A.alloc<uint32_t>((size_t)8 * (n + 1));
    B.S = A.alloc<uint32_t>(k);
    B.exoff = A.alloc<uint32_t>(p);
    B.D = A.alloc<uint32_t>(n);
    B.cnt = A.alloc<uint32_t>((size_t)p + 1);
    B.E = A.alloc<uint64_t>(std::min<size_t>(p, IPS_MAX_P) + 1);
    B.scal = A.alloc<uint32_t>(8);
    B.bst = A.alloc<uint32_t>(2 * BFS_WORDS);
    scan_reserve<uint64_t>(A, n);
    scan_reserve<uint32_t>(A, (size_t)p + 1);
}

size_t ip_workspace(uint32_t n, uint32_t m, uint32_t p, uint32_t k) {
    Arena A(nullptr, 0);
    IpBufs B;
    plan(A, n, m, p, k, B);
    return A.peak;
}

constexpr uint32_t BFS_BATCH = 8;  // BFS layers queued per host read-back

static uint32_t read_u32(const uint32_t *d, hipStream_t st) {
    uint32_t h = 0;
    read_back(&h, d, sizeof(uint32_t), st);
    return h;
}

void initial_partition(const hgp_hg &h, uint32_t k, uint32_t *part, Arena &A, hipStream_t st, int64_t W_known,
                       int64_t fill_target) {
    const uint32_t n = h.n;
    size_t mk = A.mark();
    IpBufs B;
    plan(A, n, h.m, h.p, k, B);
    const int64_t W = W_known >= 0 ? W_known : total_weight(h.vwgt, n, A, st);
    const uint64_t T = fill_target >= 0 ? (uint64_t)fill_target : (uint64_t)((W + k - 1) / k);
    // sum over nets of |e|^2: the work of expanding every pair's net
    unsigned long long sqh = 0;
    if (n && h.m) {
        unsigned long long *sq = (unsigned long long *)B.P;  // scratch until the fill
        HGP_CHECK_HIP(hipMemsetAsync(sq, 0, sizeof(unsigned long long), st));
        k_sq_sizes<<<grid_for(h.m, BLOCK, 256), BLOCK, 0, st>>>(h.pin_off, h.m, sq);
        HGP_LAUNCH_CHECK();
        read_back(&sqh, sq, sizeof(sqh), st);
    }
    // (the one-workgroup path keeps its first pair per net in exoff, which holds p words)
    const bool small = n > 0 && n <= IPS_MAX_N && h.p <= IPS_MAX_P && h.m <= h.p && sqh <= IPS_MAX_SQ;
    if (small) {
        k_ip_small<<<1, IPS_THREADS, 0, st>>>(h.pin_off, h.pins, h.inc_off, h.inc, h.vwgt, n, k, T, B.key, B.D,
                                              B.cnt, B.E, B.order, B.P, B.S, part, B.exoff, h.m);
        HGP_LAUNCH_CHECK();
        stream_sync(st);
        A.release(mk);
        return;
    }
    uint32_t *d_start = B.scal + 0, *d_cnt = B.scal + 1;
    // each net expanded once per BFS when the pairs' nets are large against
    // the pins (the extra launch per layer pays for itself)
    const bool once = sqh > 4ull * h.p;
    uint32_t *netT = once ? B.netT : nullptr, *base = once ? B.scal + 4 : nullptr;
    if (once) {
        fill<uint32_t>(B.netT, h.m, ~0u, st);
        fill<uint32_t>(base, 1, 0u, st);
    }
    HGP_CHECK_HIP(hipMemsetAsync(B.visited, 0, sizeof(uint32_t) * n, st));
    HGP_CHECK_HIP(hipMemsetAsync(B.key, 0xFF, sizeof(unsigned long long) * n, st));
    k_exoff<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.inc_off, h.inc, n, B.exoff);
    HGP_LAUNCH_CHECK();
    uint32_t pos = 0, next = 0;
    while (pos < n) {
        // next start vertex with incident nets; unreachable vertices before it join in ID order
        k_put_u32<<<1, 64, 0, st>>>(d_start, n);
        HGP_LAUNCH_CHECK();
        k_find_start<<<grid_for(n - next, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, B.visited, next, n,
                                                                               d_start);
        HGP_LAUNCH_CHECK();
        const uint32_t s = read_u32(d_start, st);
        if (s > next) {
            scan_apply<uint32_t>(A, s - next, Unvisited{B.visited, next},
                                 AppendOrder{B.visited, B.order, nullptr, next, pos}, d_cnt, st);
            const uint32_t c = read_u32(d_cnt, st);
            k_mark_range<<<grid_for(c, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.order, pos, pos + c, B.visited, B.key);
            HGP_LAUNCH_CHECK();
            pos += c;
        }
        if (s >= n) break;
        k_put_start<<<1, 64, 0, st>>>(B.order, pos, d_start, B.visited, B.bst);
        HGP_LAUNCH_CHECK();
        next = s + 1;
        // BFS layers in batches with the state in device memory (sizes are
        // bounded by n and p, layers after the last do nothing); one
        // read-back per batch tells whether the frontier has emptied.  The
        // batches of one BFS grow 1, 2, 4, ... up to BFS_BATCH layers, so a
        // small component (most of them end after a layer or two) does not
        // queue a whole batch of empty layers.
        const unsigned gT = grid_for(h.p, BLOCK, FILL_BLOCKS), gW = grid_for(n, BLOCK, FILL_BLOCKS);
        uint32_t nbatch = 1;
        for (uint32_t layer = 0;; nbatch = std::min<uint32_t>(2 * nbatch, BFS_BATCH)) {
            for (uint32_t b = 0; b < nbatch; ++b, ++layer) {
                uint32_t *cur = B.bst + (layer & 1u) * BFS_WORDS, *nxt = B.bst + ((layer + 1) & 1u) * BFS_WORDS;
                scan_apply_dn<uint32_t>(A, n, cur + BFS_F, FrontierDeg{B.order, h.inc_off, cur + BFS_FS},
                                        StoreExcl<uint32_t>{B.D}, cur + BFS_T, st);
                if (once) {
                    k_bfs_first<<<gT, BLOCK, 0, st>>>(B.D, cur, B.order, h.inc_off, h.inc, base, netT);
                    HGP_LAUNCH_CHECK();
                }
                k_bfs_keys<<<gT, BLOCK, 0, st>>>(B.D, cur, B.order, h.inc_off, h.inc, h.pin_off, h.pins, B.exoff,
                                                 B.visited, B.key, netT, base);
                HGP_LAUNCH_CHECK();
                k_bfs_winners<<<gT, BLOCK, 0, st>>>(B.D, cur, B.order, h.inc_off, h.inc, h.pin_off, h.pins,
                                                    B.exoff, B.visited, B.key, B.cnt, B.order, false, netT, base);
                HGP_LAUNCH_CHECK();
                scan_apply_dn<uint32_t>(A, h.p, cur + BFS_T, LoadArr<uint32_t>{B.cnt}, StoreExcl<uint32_t>{B.cnt},
                                        cur + BFS_W, st);
                k_bfs_winners<<<gT, BLOCK, 0, st>>>(B.D, cur, B.order, h.inc_off, h.inc, h.pin_off, h.pins,
                                                    B.exoff, B.visited, B.key, B.cnt, B.order, true, netT, base);
                HGP_LAUNCH_CHECK();
                k_bfs_mark<<<gW, BLOCK, 0, st>>>(B.order, cur, nxt, B.visited, B.key, base);
                HGP_LAUNCH_CHECK();
            }
            uint32_t hs[BFS_WORDS];
            read_back(hs, B.bst + (layer & 1u) * BFS_WORDS, sizeof(hs), st);
            if (hs[BFS_F] == 0) {
                pos = hs[BFS_POS];
                break;
            }
        }
    }
    scan_apply<uint64_t>(A, n, OrderWeight{B.order, h.vwgt}, StoreInclP{B.P}, (uint64_t *)nullptr, st);
    k_next<<<grid_for((size_t)n + 1, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.P, n, T, B.J);
    HGP_LAUNCH_CHECK();
    int levels = 0;
    while ((1u << levels) < k) ++levels;  // b < k needs `levels` bits
    for (int l = 1; l < levels; ++l) {
        k_jump<<<grid_for((size_t)n + 1, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.J + (size_t)(l - 1) * (n + 1), n,
                                                                             B.J + (size_t)l * (n + 1));
        HGP_LAUNCH_CHECK();
    }
    k_starts<<<1, 256, 0, st>>>(B.J, n, k, levels, B.S);
    HGP_LAUNCH_CHECK();
    k_assign<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(B.order, n, B.S, k, part);
    HGP_LAUNCH_CHECK();
    stream_sync(st);
    A.release(mk);
}

void project(uint32_t n, const uint32_t *cid, const uint32_t *cpart, uint32_t *part, hipStream_t st) {
    if (n == 0) return;
    k_project<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(n, cid, cpart, part);
    HGP_LAUNCH_CHECK();
}

}  // namespace hgp
