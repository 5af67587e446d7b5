// Device-wide building blocks written for gfx950 (wave64): exclusive scan
// with a fused epilogue, ordered compaction and a stable LSD radix sort of
// (key, value) pairs.  Header-only templates so each translation unit fuses
// its own input / output functors into the kernels.
#pragma once
#include "common.h"

namespace hgp {

// ---------------------------------------------------------------------------
// Exclusive scan.  A tile is BLOCK x SCAN_ITEMS values: wave w holds the run
// [w * WAVE * SCAN_ITEMS, (w + 1) * WAVE * SCAN_ITEMS) of the tile as
// SCAN_ITEMS rows of WAVE consecutive values, so every load and store of a
// wave covers 64 consecutive elements.  Element types are integers: the
// order of the additions does not change a result.
// ---------------------------------------------------------------------------
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

// Index of the value that the calling lane holds in row r of the tile at base.
__device__ inline size_t scan_elem(size_t base, int r) {
    return base + (size_t)(threadIdx.x / WAVE) * (WAVE * SCAN_ITEMS) + (size_t)r * WAVE + __lane_id();
}

// Sum of in(i) over the tile's elements below n (every thread gets it).
// Functors -------------------------------------------------------------------
template <class T>
struct LoadArr {
    const T *a;
    __device__ T operator()(size_t i) const { return a[i]; }
};
template <class T>
struct StoreExcl {
    T *out;
    __device__ void operator()(size_t i, T excl, T) const { out[i] = excl; }
};

template <class T, class In>
__device__ inline T reduce_tile(size_t base, size_t n, In in, T *lds) {
    T s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const size_t i = scan_elem(base, r);
        if (i < n) s += in(i);
    }
    s = wave_sum(s);
    if (__lane_id() == 0) lds[threadIdx.x / WAVE] = s;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int q = 0; q < BLOCK / WAVE; ++q) t += lds[q];
    __syncthreads();  // lds is reused by the caller
    return t;
}

// Calls out(i, off + exclusive prefix within the tile, in(i)) for the tile's
// elements below n; returns the tile's sum (every thread gets it).
template <class T, class In, class Out>
__device__ inline T scan_tile(size_t base, size_t n, In in, Out out, T off, T *lds) {
    const unsigned lane = __lane_id(), w = threadIdx.x / WAVE;
    T v[SCAN_ITEMS], ex[SCAN_ITEMS];
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const size_t i = scan_elem(base, r);
        v[r] = i < n ? in(i) : T(0);
    }
    T carry = 0;  // the wave's sum of the rows before
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        T x = v[r];
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const T t = __shfl_up(x, o, WAVE);
            if (lane >= (unsigned)o) x += t;
        }
        ex[r] = carry + x - v[r];
        carry += __shfl(x, WAVE - 1, WAVE);
    }
    if (lane == 0) lds[w] = carry;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < BLOCK / WAVE; ++q) {
        const T c = lds[q];
        if (q < (int)w) before += c;
        tot += c;
    }
    __syncthreads();  // lds is reused by the caller
    off += before;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const size_t i = scan_elem(base, r);
        if (i < n) out(i, off + ex[r], v[r]);
    }
    return tot;
}

template <class T, class In>
__global__ __launch_bounds__(BLOCK) void k_tile_reduce(size_t n, In in, T *tile_sum) {
    __shared__ T lds[BLOCK / WAVE];
    const T t = reduce_tile<T, In>((size_t)blockIdx.x * SCAN_TILE, n, in, lds);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = t;
}

// Single block: exclusive scan of tile sums in place; *total <- sum.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_scan_tiles(size_t ntiles, T *tile_sum, T *total) {
    __shared__ T lds[BLOCK / WAVE];
    T carry = 0;
    for (size_t base = 0; base < ntiles; base += SCAN_TILE)
        carry += scan_tile<T>(base, ntiles, LoadArr<T>{tile_sum}, StoreExcl<T>{tile_sum}, carry, lds);
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class T, class In, class Out>
__global__ __launch_bounds__(BLOCK) void k_tile_scan(size_t n, In in, Out out, const T *tile_off) {
    __shared__ T lds[BLOCK / WAVE];
    scan_tile<T, In, Out>((size_t)blockIdx.x * SCAN_TILE, n, in, out, tile_off[blockIdx.x], lds);
}

// Short inputs (at most SCAN_SMALL_TILES tiles): one block walks the tiles in
// order with a carry, one launch instead of three.
constexpr size_t SCAN_SMALL_TILES = 4;
template <class T, class In, class Out>
__global__ __launch_bounds__(BLOCK) void k_scan_small(size_t n, In in, Out out, T *total) {
    __shared__ T lds[BLOCK / WAVE];
    T carry = 0;
    for (size_t t0 = 0; t0 < n; t0 += SCAN_TILE) carry += scan_tile<T, In, Out>(t0, n, in, out, carry, lds);
    if (threadIdx.x == 0 && total) *total = carry;
}

// Medium inputs (at most SCAN_FOLD_TILES tiles): no launch for the tile
// offsets.  Every block of the scan adds up the tile sums before its own
// (L2-resident words, a few per thread); block 0 adds up all of them for
// the total.  Two launches instead of three.
constexpr size_t SCAN_FOLD_TILES = 1024;
template <class T>
__device__ inline T tile_offset(const T *tile_sum, size_t ntiles, T *total, T *lds) {
    const size_t lim = blockIdx.x == 0 ? ntiles : (size_t)blockIdx.x;
    T s = 0;
    for (size_t t = threadIdx.x; t < lim; t += BLOCK) s += tile_sum[t];
    T tot;
    block_incl_scan<T>(s, lds, &tot);
    if (blockIdx.x != 0) return tot;
    if (threadIdx.x == 0 && total) *total = tot;
    return 0;
}

template <class T, class In, class Out>
__global__ __launch_bounds__(BLOCK) void k_tile_scan_fold(size_t n, In in, Out out, const T *tile_sum,
                                                          size_t ntiles, T *total) {
    __shared__ T lds[BLOCK / WAVE];
    const T off = tile_offset<T>(tile_sum, ntiles, total, lds);
    scan_tile<T, In, Out>((size_t)blockIdx.x * SCAN_TILE, n, in, out, off, lds);
}

// out(i, exclusive_prefix, value) is called for every i < n; *total_dev gets
// the sum (may be nullptr).  Temporaries come from the arena and are released.
template <class T, class In, class Out>
void scan_apply(Arena &A, size_t n, In in, Out out, T *total_dev, hipStream_t st) {
    size_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    size_t mk = A.mark();
    T *tiles = A.alloc<T>(ntiles ? ntiles : 1);
    if (A.measure) { A.release(mk); return; }
    if (n == 0) {
        if (total_dev) HGP_CHECK_HIP(hipMemsetAsync(total_dev, 0, sizeof(T), st));
        A.release(mk);
        return;
    }
    if (ntiles <= SCAN_SMALL_TILES) {
        k_scan_small<T, In, Out><<<1, BLOCK, 0, st>>>(n, in, out, total_dev);
        HGP_LAUNCH_CHECK();
        A.release(mk);
        return;
    }
    k_tile_reduce<T, In><<<(unsigned)ntiles, BLOCK, 0, st>>>(n, in, tiles);
    HGP_LAUNCH_CHECK();
    if (ntiles <= SCAN_FOLD_TILES) {
        k_tile_scan_fold<T, In, Out><<<(unsigned)ntiles, BLOCK, 0, st>>>(n, in, out, tiles, ntiles, total_dev);
        HGP_LAUNCH_CHECK();
        A.release(mk);
        return;
    }
    k_scan_tiles<T><<<1, BLOCK, 0, st>>>(ntiles, tiles, total_dev);
    HGP_LAUNCH_CHECK();
    k_tile_scan<T, In, Out><<<(unsigned)ntiles, BLOCK, 0, st>>>(n, in, out, tiles);
    HGP_LAUNCH_CHECK();
    A.release(mk);
}

// The same scan with the element count in device memory (at most nmax), so
// that no host round trip is needed to learn the count.  The grids are fixed
// (at most DN_GRID workgroups) and stride over the tiles that the count
// reaches, so a scan costs what its count needs, not what the bound allows:
// a bound of 10^8 elements with a count of a few hundred is three short
// launches, not three launches of 50,000 workgroups.
constexpr unsigned DN_GRID = 1024;
__device__ inline size_t active_tiles(const uint32_t *n_dev) { return ((size_t)*n_dev + SCAN_TILE - 1) / SCAN_TILE; }

template <class T, class In>
__global__ __launch_bounds__(BLOCK) void k_tile_reduce_dn(const uint32_t *n_dev, In in, T *tile_sum) {
    __shared__ T lds[BLOCK / WAVE];
    const size_t n = *n_dev, nt = active_tiles(n_dev);
    for (size_t t = blockIdx.x; t < nt; t += gridDim.x) {  // uniform per block
        const T v = reduce_tile<T, In>(t * SCAN_TILE, n, in, lds);
        if (threadIdx.x == 0) tile_sum[t] = v;
        __syncthreads();  // lds is reused by the next tile
    }
}

// Single block: exclusive scan of the active tile sums in place; *total <- sum.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_scan_tiles_dn(const uint32_t *n_dev, T *tile_sum, T *total) {
    __shared__ T lds[BLOCK / WAVE];
    const size_t nt = active_tiles(n_dev);
    T carry = 0;
    for (size_t base = 0; base < nt; base += SCAN_TILE)
        carry += scan_tile<T>(base, nt, LoadArr<T>{tile_sum}, StoreExcl<T>{tile_sum}, carry, lds);
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class T, class In, class Out>
__global__ __launch_bounds__(BLOCK) void k_tile_scan_dn(const uint32_t *n_dev, In in, Out out, const T *tile_off) {
    __shared__ T lds[BLOCK / WAVE];
    const size_t n = *n_dev, nt = active_tiles(n_dev);
    for (size_t t = blockIdx.x; t < nt; t += gridDim.x) {  // uniform per block
        scan_tile<T, In, Out>(t * SCAN_TILE, n, in, out, tile_off[t], lds);
        __syncthreads();
    }
}

template <class T, class In, class Out>
__global__ __launch_bounds__(BLOCK) void k_scan_small_dn(const uint32_t *n_dev, In in, Out out, T *total) {
    __shared__ T lds[BLOCK / WAVE];
    const size_t n = *n_dev;
    T carry = 0;
    for (size_t t0 = 0; t0 < n; t0 += SCAN_TILE) carry += scan_tile<T, In, Out>(t0, n, in, out, carry, lds);
    if (threadIdx.x == 0 && total) *total = carry;
}

// With the count on the device the single-block walk covers only the tiles
// the count reaches, so it is taken up to twice as many tiles of the bound.
constexpr size_t SCAN_SMALL_TILES_DN = 2 * SCAN_SMALL_TILES;
template <class T, class In, class Out>
void scan_apply_dn(Arena &A, size_t nmax, const uint32_t *n_dev, In in, Out out, T *total_dev, hipStream_t st) {
    const size_t ntiles = (nmax + SCAN_TILE - 1) / SCAN_TILE;
    size_t mk = A.mark();
    T *tiles = A.alloc<T>(ntiles ? ntiles : 1);
    if (A.measure) { A.release(mk); return; }
    if (ntiles <= SCAN_SMALL_TILES_DN) {
        k_scan_small_dn<T, In, Out><<<1, BLOCK, 0, st>>>(n_dev, in, out, total_dev);
        HGP_LAUNCH_CHECK();
        A.release(mk);
        return;
    }
    const unsigned g = (unsigned)std::min<size_t>(ntiles, DN_GRID);
    k_tile_reduce_dn<T, In><<<g, BLOCK, 0, st>>>(n_dev, in, tiles);
    HGP_LAUNCH_CHECK();
    k_scan_tiles_dn<T><<<1, BLOCK, 0, st>>>(n_dev, tiles, total_dev);
    HGP_LAUNCH_CHECK();
    k_tile_scan_dn<T, In, Out><<<g, BLOCK, 0, st>>>(n_dev, in, out, tiles);
    HGP_LAUNCH_CHECK();
    A.release(mk);
}

// Size-only reservation of scan_apply's temporaries (never launches).
template <class T>
inline void scan_reserve(Arena &A, size_t n) {
    size_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    size_t mk = A.mark();
    A.alloc<T>(ntiles ? ntiles : 1);
    A.release(mk);
}


// Exclusive scan of an array into another (may alias): out[i] = sum a[0:i].
template <class T>
void exclusive_scan(Arena &A, const T *a, T *out, size_t n, T *total_dev, hipStream_t st) {
    scan_apply<T>(A, n, LoadArr<T>{a}, StoreExcl<T>{out}, total_dev, st);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs; 8-bit digits.
// ---------------------------------------------------------------------------
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = BLOCK * RS_ITEMS;

// Digit of every valid lane; `match` gets the lanes of the wave holding the
// same digit (eight ballots).
__device__ inline uint64_t digit_match(bool valid, uint32_t d) {
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t vote = __ballot(bit);
        match &= bit ? vote : ~vote;
    }
    return match;
}

// Per-tile digit histogram; all RS_ITEMS keys of a thread are loaded first.
template <class K>
__global__ __launch_bounds__(BLOCK) void k_rs_hist(const K *keys, size_t n, const uint32_t *n_dev, int shift,
                                                   uint32_t ntiles, uint32_t *counts) {
    __shared__ uint32_t h[256];
    if (n_dev && (size_t)*n_dev < n) n = *n_dev;
    h[threadIdx.x] = 0;
    const size_t base = (size_t)blockIdx.x * RS_TILE;
    uint32_t dg[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const size_t i = base + (size_t)r * BLOCK + threadIdx.x;
        dg[r] = i < n ? ((uint32_t)(keys[i] >> shift) & 0xFFu) : 256u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const bool valid = dg[r] < 256u;
        const uint32_t d = dg[r] & 0xFFu;
        const uint64_t match = digit_match(valid, d);  // one LDS atomic per distinct digit of the wave
        if (valid && (match & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(match));
    }
    __syncthreads();
    counts[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: the tile is first ordered by digit in LDS
// (rank within the digit = earlier rounds, earlier waves, earlier lanes),
// then written out position by position, so the elements of a digit bucket
// leave as one contiguous run instead of single scattered words.
template <class K>
__global__ __launch_bounds__(BLOCK) void k_rs_scatter(const K *keys, const uint32_t *vals, K *keys_out,
                                                      uint32_t *vals_out, size_t n, const uint32_t *n_dev,
                                                      int shift, uint32_t ntiles, const uint32_t *offsets) {
    __shared__ K skey[RS_TILE];
    __shared__ uint32_t sval[RS_TILE];
    __shared__ uint32_t wcnt[BLOCK / WAVE][256];
    __shared__ uint32_t run[256];   // elements of each digit in the rounds so far
    __shared__ uint32_t tpre[256];  // exclusive prefix of the tile's digit counts
    __shared__ uint32_t gout[256];  // where the tile's bucket of each digit starts in the output
    __shared__ uint32_t wsum[BLOCK / WAVE];
    const unsigned tid = threadIdx.x, w = tid / WAVE;
    if (n_dev && (size_t)*n_dev < n) n = *n_dev;
    gout[tid] = offsets[(size_t)tid * ntiles + blockIdx.x];
    run[tid] = 0;
    const size_t tbase = (size_t)blockIdx.x * RS_TILE;
    K kr[RS_ITEMS];
    uint32_t vr[RS_ITEMS], rk[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const size_t i = tbase + (size_t)r * BLOCK + tid;
        kr[r] = i < n ? keys[i] : K(0);
        vr[r] = i < n ? vals[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
#pragma unroll
        for (int q = 0; q < BLOCK / WAVE; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        const bool valid = tbase + (size_t)r * BLOCK + tid < n;
        const uint32_t d = (uint32_t)(kr[r] >> shift) & 0xFFu;
        const uint64_t match = digit_match(valid, d);
        const uint32_t rank = (uint32_t)__popcll(match & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(match);
        __syncthreads();
        uint32_t pos = run[d] + rank;
        for (unsigned q = 0; q < w; ++q) pos += wcnt[q][d];
        rk[r] = pos;
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < BLOCK / WAVE; ++q) add += wcnt[q][tid];
        run[tid] += add;
    }
    __syncthreads();
    const uint32_t c = run[tid];
    uint32_t tot;
    const uint32_t incl = block_incl_scan<uint32_t>(c, wsum, &tot);
    tpre[tid] = incl - c;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        if (tbase + (size_t)r * BLOCK + tid < n) {
            const uint32_t p = tpre[(uint32_t)(kr[r] >> shift) & 0xFFu] + rk[r];
            skey[p] = kr[r];
            sval[p] = vr[r];
        }
    }
    __syncthreads();
    const uint32_t cnt = tbase >= n ? 0u : (uint32_t)(n - tbase < (size_t)RS_TILE ? n - tbase : (size_t)RS_TILE);
    for (uint32_t p = tid; p < cnt; p += BLOCK) {
        const K key = skey[p];
        const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
        const size_t o = (size_t)gout[d] + (p - tpre[d]);
        keys_out[o] = key;
        vals_out[o] = sval[p];
    }
}

// Sorts n pairs by bits [begin_bit, end_bit) of the key, stably.  The sorted
// data ends in (*keys_io, *vals_io), which may be swapped with the alternate
// buffers given.  With n_dev, the pairs sorted are the first min(n, *n_dev)
// (a count the stream produces): n only sizes the launches.
template <class K>
void radix_sort_pairs(Arena &A, K **keys_io, uint32_t **vals_io, K *keys_alt, uint32_t *vals_alt,
                      size_t n, int begin_bit, int end_bit, hipStream_t st, const uint32_t *n_dev = nullptr) {
    uint32_t ntiles = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
    size_t mk = A.mark();
    uint32_t *counts = A.alloc<uint32_t>((size_t)256 * (ntiles ? ntiles : 1));
    scan_reserve<uint32_t>(A, (size_t)256 * (ntiles ? ntiles : 1));
    if (A.measure || n == 0) { A.release(mk); return; }
    K *kin = *keys_io, *kout = keys_alt;
    uint32_t *vin = *vals_io, *vout = vals_alt;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        k_rs_hist<K><<<ntiles, BLOCK, 0, st>>>(kin, n, n_dev, shift, ntiles, counts);
        HGP_LAUNCH_CHECK();
        exclusive_scan<uint32_t>(A, counts, counts, (size_t)256 * ntiles, nullptr, st);
        k_rs_scatter<K><<<ntiles, BLOCK, 0, st>>>(kin, vin, kout, vout, n, n_dev, shift, ntiles, counts);
        HGP_LAUNCH_CHECK();
        K *tk = kin; kin = kout; kout = tk;
        uint32_t *tv = vin; vin = vout; vout = tv;
    }
    *keys_io = kin;
    *vals_io = vin;
    A.release(mk);
}

// Size-only reservation of radix_sort_pairs' temporaries (never launches).
inline void sort_reserve(Arena &A, size_t n) {
    size_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    size_t mk = A.mark();
    A.alloc<uint32_t>((size_t)256 * (ntiles ? ntiles : 1));
    scan_reserve<uint32_t>(A, (size_t)256 * (ntiles ? ntiles : 1));
    A.release(mk);
}

inline int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T *p, size_t n, T v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
inline void fill(T *p, size_t n, T v, hipStream_t st) {
    if (n == 0) return;
    k_fill<T><<<grid_for(n, BLOCK * 4, FILL_BLOCKS), BLOCK, 0, st>>>(p, n, v);
    HGP_LAUNCH_CHECK();
}

template <class T>
__global__ void k_iota(T *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = (T)i;
}

}  // namespace hgp
