// Internal helpers of the gfx950 library: arena workspace, launch checking,
// wave64 primitives and the seeded hash.  Not part of the public ABI.
#pragma once
#include <initializer_list>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include "../../include/hgp.h"

namespace hgp {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int WAVE = 64;
constexpr int BLOCK = 256;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
struct Error {
    hgp_status code;
};

#define HGP_CHECK_HIP(expr)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) throw ::hgp::Error{HGP_E_DEVICE}; \
    } while (0)

// Host waits for a stream.  By default they spin (lowest latency for a single
// caller).  The worker threads of a partition server set blocking_waits: the
// wait then sleeps in the driver, so that many waiting lanes do not occupy
// the host cores that the launching lanes need.
inline thread_local bool blocking_waits = false;
void stream_sync(hipStream_t st);

// Pinned host words of the calling thread (MAILBOX_WORDS of them): a counter
// copied there with hipMemcpyAsync is valid after the next stream_sync of
// that stream, so a read-back can wait for a sync the caller needs anyway.
constexpr int MAILBOX_WORDS = 16;
uint32_t *host_mailbox();

// Reads device memory into host memory and waits for the stream.  The copies
// land in the calling thread's pinned staging buffer (STAGE_BYTES, allocated
// on first use), so they queue behind one wait: a copy to pageable memory is a
// host round trip of its own.  A read larger than what is left of the buffer
// goes straight to its destination.  Every destination holds its bytes on
// return.  It allocates the buffer on a thread's first call unless
// may_allocate is false; then a thread without one copies straight to the
// destinations (the LP driver, which the allocation-free entry point runs,
// never allocates).
struct HostRead {
    void *dst;
    const void *src;
    size_t bytes;
};
constexpr size_t STAGE_BYTES = 64 * 1024;
void read_back(std::initializer_list<HostRead> reads, hipStream_t st, bool may_allocate = true);
inline void read_back(void *dst, const void *src, size_t bytes, hipStream_t st, bool may_allocate = true) {
    read_back({{dst, src, bytes}}, st, may_allocate);
}

#define HGP_LAUNCH_CHECK() HGP_CHECK_HIP(hipGetLastError())

#define HGP_REQUIRE(cond, code)                 \
    do {                                        \
        if (!(cond)) throw ::hgp::Error{code};  \
    } while (0)

// ---------------------------------------------------------------------------
// Workspace arena: bump allocation over the caller's buffer.  With base ==
// nullptr it only measures (used by hgp_workspace_bytes), so the size query
// and the real allocation run the same code.
// ---------------------------------------------------------------------------
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t top = 0;
    size_t peak = 0;
    bool measure = false;

    Arena(void *b, size_t c) : base((char *)b), cap(c), measure(b == nullptr) {}

    template <class T>
    T *alloc(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        size_t off = top;
        top += bytes;
        if (top > peak) peak = top;
        if (measure) return nullptr;
        if (top > cap) throw Error{HGP_E_WORKSPACE};
        return (T *)(base + off);
    }
    size_t mark() const { return top; }
    // bytes still free (unbounded when only measuring)
    size_t remaining() const { return measure ? ~size_t(0) : (cap > top ? cap - top : 0); }
    void release(size_t m) { top = m; }
};

inline unsigned grid_for(size_t work, int per_block, unsigned max_blocks = 65535u * 4) {
    size_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (unsigned)g;
}

// Number of blocks of a grid-stride kernel that fill the chip (256 CUs).
constexpr unsigned FILL_BLOCKS = 2048;
// Grid cap of kernels that end in one device-scope atomic per workgroup on a
// few shared addresses (such atomics are serialised).
constexpr unsigned REDUCE_BLOCKS = 256;

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

// H(seed, purpose, level, it, x) with mseed = mix64(seed) precomputed.
__host__ __device__ inline uint64_t tag_hash(uint64_t mseed, uint32_t purpose, uint32_t level,
                                             uint32_t it, uint32_t x) {
    uint64_t tag = (uint64_t)((purpose & 0xFFu) | ((level & 0xFFu) << 8) | ((it & 0xFFFFu) << 16));
    return mix64(mseed ^ ((tag << 32) | (uint64_t)x));
}

__device__ inline unsigned lane_id() { return __lane_id(); }

__device__ inline uint64_t lanemask_lt() {
    unsigned l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Wave-level ordering point for LDS traffic shared between lanes of a wave.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Inclusive block scan of one value per thread (blockDim == BLOCK).
template <class T>
__device__ inline T block_incl_scan(T v, T *lds /*[BLOCK/WAVE]*/, T *total) {
    unsigned l = __lane_id();
    unsigned w = threadIdx.x / WAVE;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (l >= (unsigned)o) v += t;
    }
    if (l == 63) lds[w] = v;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / WAVE; ++i) {
        T s = lds[i];
        if (i < (int)w) off += s;
        tot += s;
    }
    __syncthreads();
    if (total) *total = tot;
    return v + off;
}

// Inclusive scan over a block of NT threads; *total (per thread) <- block sum.
template <class T, int NT>
__device__ inline T block_incl_scan_n(T v, T *lds /*[NT/WAVE]*/, T *total) {
    unsigned l = __lane_id();
    unsigned w = threadIdx.x / WAVE;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (l >= (unsigned)o) v += t;
    }
    if (l == 63) lds[w] = v;
    __syncthreads();
    T off = 0, tot = 0;
    for (int i = 0; i < NT / WAVE; ++i) {
        T s = lds[i];
        if (i < (int)w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return v + off;
}

// Atomic add for int64 in global memory.
// XCD-aware split of the index range [0, count) over a grid of nblk
// workgroups.  gfx950 dispatches workgroup b to XCD b % 8, and each XCD has
// its own L2, so XCD x takes the x-th contiguous eighth of the range and its
// workgroups (wi = 0 .. nw-1) stride over that eighth.  Neighbouring items
// (which share cache lines and, in the meshes and locally numbered inputs,
// incident nets) then stay in one L2.  Any grid size is valid.
struct XcdSlice {
    uint32_t lo, hi, wi, nw;
};
__device__ inline XcdSlice xcd_slice(uint32_t blk, uint32_t nblk, uint32_t count) {
    if (nblk < 8) return {0u, count, blk, nblk};
    const uint32_t x = blk % 8;
    return {(uint32_t)((uint64_t)count * x / 8), (uint32_t)((uint64_t)count * (x + 1) / 8), blk / 8,
            nblk / 8 + (x < nblk % 8 ? 1u : 0u)};
}

__device__ inline void atomic_add_i64(int64_t *p, int64_t v) {
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// Device-scope atomics on one address are serialised (about 80 million per
// second on the whole chip), so accumulators that every workgroup feeds are
// spread over SPREAD slots 128 bytes apart: a workgroup adds into slot
// blockIdx.x % SPREAD and the reader sums the slots.
constexpr uint32_t SPREAD = 64;
constexpr uint32_t SPREAD_I64 = 16;  // slot stride in int64 (128 bytes)
constexpr uint32_t SPREAD_U32 = 32;  // slot stride in uint32 (128 bytes)
__device__ inline void spread_add_i64(int64_t *acc, int64_t v) {
    atomicAdd((unsigned long long *)&acc[(blockIdx.x % SPREAD) * SPREAD_I64], (unsigned long long)v);
}
// Sum of a spread accumulator by one wave (lane i reads slot i).
__device__ inline int64_t spread_total_wave(const int64_t *acc) {
    int64_t x = acc[(__lane_id() % SPREAD) * SPREAD_I64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ inline uint32_t warp_agg_append(uint32_t *counter, bool pred) {
    // Returns the slot of this lane in an append-only list (only valid if pred).
    uint64_t m = __ballot(pred);
    if (m == 0) return NONE;
    int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(m & lanemask_lt());
}

}  // namespace hgp
