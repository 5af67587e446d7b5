// Greedy initial partition of the coarsest level (a simple deterministic
// method; the paper's portfolio of Sec. 5 is not part of this path) and the
// projection step of uncoarsening (Sec. 3).
//
// Order: breadth-first from the smallest unvisited vertex, neighbours taken
// in ascending incident-net order and, inside a net, ascending pin order.
// One workgroup computes it exactly, one BFS level at a time: every
// occurrence of an unvisited vertex in the expansion of the frontier gets the
// key (frontier position, offset in that vertex's expansion); the vertex
// joins the next frontier at its smallest key, and the new frontier is laid
// out in key order by a block scan (frontier vertices are processed in order
// and each one's occurrences in order, so key order = thread order).
// Fill: block b covers positions [S_b, S_{b+1}) of the order, where
// S_{b+1} = 1 + first i >= S_b with weight(S_b..i) >= ceil(c(V)/k); the S_b
// are found by pointer doubling over next(s), the last block takes the rest.
#include "prims.h"
#include "kernels.h"

namespace hgp {

constexpr int BFS_THREADS = 1024;

__device__ inline uint64_t aload(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(BFS_THREADS) void k_bfs(const uint32_t *pin_off, const uint32_t *pins,
                                                     const uint32_t *inc_off, const uint32_t *inc, uint32_t n,
                                                     uint32_t *order, uint32_t *visited, unsigned long long *key) {
    __shared__ uint32_t s_found;
    __shared__ uint32_t wsum[BFS_THREADS / WAVE];
    const uint32_t tid = threadIdx.x;
    uint32_t pos = 0, next_start = 0;
    while (pos < n) {
        // smallest unvisited vertex >= next_start
        for (uint32_t base = next_start;; base += BFS_THREADS) {
            if (tid == 0) s_found = NONE;
            __syncthreads();
            uint32_t idx = base + tid;
            if (idx < n && __hip_atomic_load(&visited[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
                atomicMin(&s_found, idx);
            __syncthreads();
            uint32_t f = s_found;
            __syncthreads();
            if (f != NONE || base + BFS_THREADS >= n) {
                next_start = f;
                break;
            }
        }
        const uint32_t start = next_start;  // exists because pos < n
        if (start == NONE) break;            // unreachable for a consistent input
        next_start = start + 1;
        if (tid == 0) {
            __hip_atomic_store(&visited[start], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            order[pos] = start;
        }
        uint32_t fstart = pos, fend = pos + 1;
        pos += 1;
        __syncthreads();
        while (fstart < fend) {
            // phase 1: smallest key of every unvisited vertex reached
            for (uint32_t c = fstart; c < fend; c += BFS_THREADS) {
                uint32_t fi = c + tid;
                if (fi < fend) {
                    uint32_t v = order[fi];
                    uint64_t hi = (uint64_t)(fi - fstart) << 32;
                    uint32_t off = 0;
                    for (uint32_t j = inc_off[v]; j < inc_off[v + 1]; ++j) {
                        uint32_t e = inc[j];
                        for (uint32_t q = pin_off[e]; q < pin_off[e + 1]; ++q, ++off) {
                            uint32_t w = pins[q];
                            if (__hip_atomic_load(&visited[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
                                atomicMin(&key[w], (unsigned long long)(hi | off));
                        }
                    }
                }
            }
            __threadfence();
            __syncthreads();
            // phase 2: winners appended in key order
            uint32_t newpos = pos;
            for (uint32_t c = fstart; c < fend; c += BFS_THREADS) {
                uint32_t fi = c + tid;
                uint32_t cnt = 0;
                uint32_t v = 0;
                uint64_t hi = (uint64_t)(fi - fstart) << 32;
                if (fi < fend) {
                    v = order[fi];
                    uint32_t off = 0;
                    for (uint32_t j = inc_off[v]; j < inc_off[v + 1]; ++j) {
                        uint32_t e = inc[j];
                        for (uint32_t q = pin_off[e]; q < pin_off[e + 1]; ++q, ++off) {
                            uint32_t w = pins[q];
                            if (__hip_atomic_load(&visited[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                                aload((const uint64_t *)&key[w]) == (hi | off))
                                ++cnt;
                        }
                    }
                }
                uint32_t tot;
                uint32_t incl = block_incl_scan_n<uint32_t, BFS_THREADS>(cnt, wsum, &tot);
                uint32_t wpos = newpos + incl - cnt;
                if (fi < fend && cnt) {
                    uint32_t off = 0;
                    for (uint32_t j = inc_off[v]; j < inc_off[v + 1]; ++j) {
                        uint32_t e = inc[j];
                        for (uint32_t q = pin_off[e]; q < pin_off[e + 1]; ++q, ++off) {
                            uint32_t w = pins[q];
                            if (__hip_atomic_load(&visited[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                                aload((const uint64_t *)&key[w]) == (hi | off))
                                order[wpos++] = w;
                        }
                    }
                }
                newpos += tot;
                __syncthreads();
            }
            __threadfence();
            __syncthreads();
            // phase 3: mark the new frontier visited, reset keys
            for (uint32_t i = pos + tid; i < newpos; i += BFS_THREADS) {
                uint32_t w = order[i];
                __hip_atomic_store(&visited[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicExch(&key[w], ~0ull);
            }
            __threadfence();
            __syncthreads();
            fstart = fend;
            fend = newpos;
            pos = newpos;
        }
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

struct IpBufs {
    uint32_t *order, *visited, *J, *S;
    unsigned long long *key;
    uint64_t *P;
};

static void plan(Arena &A, uint32_t n, uint32_t k, IpBufs &B) {
    B.order = A.alloc<uint32_t>(n);
    B.visited = A.alloc<uint32_t>(n);
    B.key = A.alloc<unsigned long long>(n);
    B.P = A.alloc<uint64_t>(n);
    B.J = A.alloc<uint32_t>((size_t)8 * (n + 1));
    B.S = A.alloc<uint32_t>(k);
    scan_reserve<uint64_t>(A, n);
}

size_t ip_workspace(uint32_t n, uint32_t k) {
    Arena A(nullptr, 0);
    IpBufs B;
    plan(A, n, k, B);
    return A.peak;
}

void initial_partition(const hgp_hg &h, uint32_t k, uint32_t *part, Arena &A, hipStream_t st) {
    const uint32_t n = h.n;
    size_t mk = A.mark();
    IpBufs B;
    plan(A, n, k, B);
    const int64_t W = total_weight(h.vwgt, n, A, st);
    const uint64_t T = (uint64_t)((W + k - 1) / k);
    HGP_CHECK_HIP(hipMemsetAsync(B.visited, 0, sizeof(uint32_t) * n, st));
    HGP_CHECK_HIP(hipMemsetAsync(B.key, 0xFF, sizeof(unsigned long long) * n, st));
    k_bfs<<<1, BFS_THREADS, 0, st>>>(h.pin_off, h.pins, h.inc_off, h.inc, n, B.order, B.visited, B.key);
    HGP_LAUNCH_CHECK();
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
    HGP_CHECK_HIP(hipStreamSynchronize(st));
    A.release(mk);
}

void project(uint32_t n, const uint32_t *cid, const uint32_t *cpart, uint32_t *part, hipStream_t st) {
    if (n == 0) return;
    k_project<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(n, cid, cpart, part);
    HGP_LAUNCH_CHECK();
}

}  // namespace hgp
