// Segmented ascending sort of uint32 values inside CSR segments, with an
// optional de-duplication that moves the distinct values to the front of
// each segment and records their count.  Four tiers by segment length:
//   <= 16    one thread per segment, a sorting network in registers;
//   <= 64    one wave per segment, a value per lane, bitonic sort by shuffles;
//   <= 4096  one block per segment, bitonic sort in LDS;
//   larger   all such segments together through the device radix sort on
//            (segment rank, value) keys, then a block per segment compacts.
#pragma once
#include "prims.h"

namespace hgp {

constexpr uint32_t SEG_SMALL = 16;
constexpr uint32_t SEG_WAVE = 64;
constexpr uint32_t SEG_MED = 4096;

__device__ inline void cswap(uint32_t &a, uint32_t &b) {
    uint32_t x = a < b ? a : b;
    uint32_t y = a < b ? b : a;
    a = x;
    b = y;
}

// Bitonic sorting network on 16 registers (ascending).
__device__ inline void sort16(uint32_t (&r)[16]) {
#pragma unroll
    for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                int l = i ^ j;
                if (l > i) {
                    if ((i & k) == 0) cswap(r[i], r[l]);
                    else cswap(r[l], r[i]);
                }
            }
        }
    }
}

// Small segments: sort (+unique).  Segments longer than SEG_MED and up to
// SEG_MED are appended to the large / medium lists; segments of the wave tier
// are only flagged (a plain store): k_seg_wave finds them itself, since they
// can be as many as the segments and a shared append counter costs one
// serialised device-scope atomic per wave.
__global__ void k_seg_small(const uint32_t *off, uint32_t nseg, uint32_t *data, bool uniq, uint32_t *usize,
                            uint32_t *med, uint32_t *nmed, uint32_t *large, uint32_t *nlarge, uint32_t *wflag) {
    for (uint32_t s0 = blockIdx.x * blockDim.x; s0 < nseg; s0 += gridDim.x * blockDim.x) {
        uint32_t s = s0 + threadIdx.x;
        bool act = s < nseg;
        uint32_t b = act ? off[s] : 0, len = act ? off[s + 1] - b : 0;
        bool iswave = act && len > SEG_SMALL && len <= SEG_WAVE;
        bool ismed = act && len > SEG_WAVE && len <= SEG_MED;
        bool islarge = act && len > SEG_MED;
        if (__ballot(iswave) && __lane_id() == 0) *wflag = 1u;
        uint32_t pm = warp_agg_append(nmed, ismed);
        if (ismed) med[pm] = s;
        uint32_t pl = warp_agg_append(nlarge, islarge);
        if (islarge) large[pl] = s;
        if (!act || len > SEG_SMALL) continue;
        uint32_t r[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = (uint32_t)i < len ? data[b + i] : 0xFFFFFFFFu;
        sort16(r);
        if (!uniq) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if ((uint32_t)i < len) data[b + i] = r[i];
        } else {
            uint32_t w = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if ((uint32_t)i < len && (i == 0 || r[i] != r[i - 1])) {
                    data[b + w] = r[i];
                    ++w;
                }
            }
            usize[s] = w;
        }
    }
}

// Segments of SEG_SMALL+1 .. SEG_WAVE values: one wave each, a value per lane,
// bitonic sort by shuffles; the distinct values are compacted by a ballot.
// A wave takes 64 consecutive segments at a time and sorts those of the tier.
__global__ __launch_bounds__(BLOCK) void k_seg_wave(const uint32_t *off, uint32_t nseg, uint32_t *data, bool uniq,
                                                    uint32_t *usize) {
    const uint32_t lane = __lane_id();
    const uint32_t wid = (blockIdx.x * BLOCK + threadIdx.x) / WAVE, nw = gridDim.x * BLOCK / WAVE;
    for (uint32_t s0 = wid * WAVE; s0 < nseg; s0 += nw * WAVE) {
      const uint32_t sl = s0 + lane;
      const uint32_t ll = sl < nseg ? off[sl + 1] - off[sl] : 0;
      uint64_t todo = __ballot(ll > SEG_SMALL && ll <= SEG_WAVE);
      while (todo) {
        const uint32_t s = s0 + (uint32_t)(__ffsll((long long)todo) - 1);
        todo &= todo - 1;
        const uint32_t b = off[s], len = off[s + 1] - b;
        uint32_t x = lane < len ? data[b + lane] : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                const uint32_t y = __shfl_xor(x, (int)j, 64);
                const bool up = (lane & k) == 0, lower = (lane & j) == 0;
                x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
            }
        }
        if (!uniq) {
            if (lane < len) data[b + lane] = x;
        } else {
            const uint32_t prev = __shfl_up(x, 1, 64);
            const bool keep = lane < len && (lane == 0 || x != prev);
            const uint64_t mk = __ballot(keep);
            if (keep) data[b + (uint32_t)__popcll(mk & lanemask_lt())] = x;
            if (lane == 0) usize[s] = (uint32_t)__popcll(mk);
        }
      }
    }
}

// Medium segments: one block each, bitonic sort of up to 4096 values in LDS.
__global__ __launch_bounds__(BLOCK) void k_seg_med(const uint32_t *off, const uint32_t *list, uint32_t count,
                                                   uint32_t *data, bool uniq, uint32_t *usize) {
    __shared__ uint32_t v[SEG_MED];
    __shared__ uint32_t wsum[BLOCK / WAVE];
    for (uint32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        uint32_t s = list[idx];
        uint32_t b = off[s], len = off[s + 1] - b;
        uint32_t P = 32;
        while (P < len) P <<= 1;
        for (uint32_t i = threadIdx.x; i < P; i += BLOCK) v[i] = i < len ? data[b + i] : 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = threadIdx.x; i < P; i += BLOCK) {
                    uint32_t l = i ^ j;
                    if (l > i) {
                        uint32_t x = v[i], y = v[l];
                        bool up = (i & k) == 0;
                        if ((x > y) == up) { v[i] = y; v[l] = x; }
                    }
                }
                __syncthreads();
            }
        }
        if (!uniq) {
            for (uint32_t i = threadIdx.x; i < len; i += BLOCK) data[b + i] = v[i];
        } else {
            // stable compaction of first occurrences, chunk by chunk
            uint32_t carry = 0;
            for (uint32_t c0 = 0; c0 < len; c0 += BLOCK) {
                uint32_t i = c0 + threadIdx.x;
                uint32_t keep = (i < len && (i == 0 || v[i] != v[i - 1])) ? 1u : 0u;
                uint32_t tot;
                uint32_t incl = block_incl_scan<uint32_t>(keep, wsum, &tot);
                if (keep) data[b + carry + incl - 1] = v[i];
                carry += tot;
            }
            if (threadIdx.x == 0) usize[s] = carry;
        }
        __syncthreads();
    }
}

// Large segments: gather (rank, value) keys.
__global__ void k_seg_large_gather(const uint32_t *off, const uint32_t *list, uint32_t count, const uint32_t *data,
                                   const uint64_t *pos /*exclusive offsets of the large segments*/, uint64_t *keys,
                                   uint32_t *vals) {
    for (uint32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        uint32_t s = list[idx];
        uint32_t b = off[s], len = off[s + 1] - b;
        uint64_t p0 = pos[idx];
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
            keys[p0 + i] = ((uint64_t)idx << 32) | data[b + i];
            vals[p0 + i] = 0;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_seg_large_scatter(const uint32_t *off, const uint32_t *list,
                                                             uint32_t count, uint32_t *data, const uint64_t *pos,
                                                             const uint64_t *keys, bool uniq, uint32_t *usize) {
    __shared__ uint32_t wsum[BLOCK / WAVE];
    for (uint32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        uint32_t s = list[idx];
        uint32_t b = off[s], len = off[s + 1] - b;
        uint64_t p0 = pos[idx];
        if (!uniq) {
            for (uint32_t i = threadIdx.x; i < len; i += BLOCK) data[b + i] = (uint32_t)keys[p0 + i];
        } else {
            uint32_t carry = 0;
            for (uint32_t c0 = 0; c0 < len; c0 += BLOCK) {
                uint32_t i = c0 + threadIdx.x;
                uint32_t val = i < len ? (uint32_t)keys[p0 + i] : 0;
                uint32_t keep = (i < len && (i == 0 || val != (uint32_t)keys[p0 + i - 1])) ? 1u : 0u;
                uint32_t tot;
                uint32_t incl = block_incl_scan<uint32_t>(keep, wsum, &tot);
                if (keep) data[b + carry + incl - 1] = val;
                carry += tot;
            }
            if (threadIdx.x == 0) usize[s] = carry;
        }
        __syncthreads();
    }
}

struct LargeLen {
    const uint32_t *off, *list;
    __device__ uint64_t operator()(size_t i) const { uint32_t s = list[i]; return off[s + 1] - off[s]; }
};

struct SegSortBufs {
    uint32_t *med, *large, *scal;
    uint64_t *pos, *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
};

// Workspace for segments holding at most `total` values.
inline void segsort_plan(Arena &A, uint32_t nseg, size_t total, SegSortBufs &B) {
    B.med = A.alloc<uint32_t>(nseg);
    B.large = A.alloc<uint32_t>(total / SEG_MED + 1);
    B.scal = A.alloc<uint32_t>(6);
    B.pos = A.alloc<uint64_t>(total / SEG_MED + 2);
    B.keys = A.alloc<uint64_t>(total);
    B.keys_alt = A.alloc<uint64_t>(total);
    B.vals = A.alloc<uint32_t>(total);
    B.vals_alt = A.alloc<uint32_t>(total);
    sort_reserve(A, total);
    scan_reserve<uint64_t>(A, total / SEG_MED + 1);
}

// Sorts (and with uniq, de-duplicates) every segment.  Syncs the stream.
// tiers[0], tiers[1] (host) receive the numbers of segments of the block and
// device-wide tiers (B.med and B.large list them).
inline void segmented_sort(Arena &A, const SegSortBufs &B, const uint32_t *off, uint32_t nseg, uint32_t *data,
                           bool uniq, uint32_t *usize, uint32_t *tiers, hipStream_t st) {
    tiers[0] = tiers[1] = 0;
    if (nseg == 0) {
        stream_sync(st);
        return;
    }
    HGP_CHECK_HIP(hipMemsetAsync(B.scal, 0, sizeof(uint32_t) * 6, st));
    k_seg_small<<<grid_for(nseg, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(off, nseg, data, uniq, usize, B.med, B.scal,
                                                                     B.large, B.scal + 1, B.scal + 4);
    HGP_LAUNCH_CHECK();
    uint32_t cnt[5];
    read_back(cnt, B.scal, sizeof(cnt), st);
    tiers[0] = cnt[0];
    tiers[1] = cnt[1];
    if (cnt[4]) {  // some segment of the wave tier
        k_seg_wave<<<grid_for(nseg, BLOCK, 8192), BLOCK, 0, st>>>(off, nseg, data, uniq, usize);
        HGP_LAUNCH_CHECK();
    }
    if (cnt[0]) {
        k_seg_med<<<grid_for(cnt[0], 1, 4096), BLOCK, 0, st>>>(off, B.med, cnt[0], data, uniq, usize);
        HGP_LAUNCH_CHECK();
    }
    if (cnt[1]) {
        uint32_t nl = cnt[1];
        uint64_t total = 0;
        uint64_t *tot_dev = (uint64_t *)(B.scal + 2);
        scan_apply<uint64_t>(A, nl, LargeLen{off, B.large}, StoreExcl<uint64_t>{B.pos}, tot_dev, st);
        read_back(&total, tot_dev, sizeof(uint64_t), st);
        k_seg_large_gather<<<grid_for(nl, 1, 4096), BLOCK, 0, st>>>(off, B.large, nl, data, B.pos, B.keys, B.vals);
        HGP_LAUNCH_CHECK();
        uint64_t *kk = B.keys;
        uint32_t *vv = B.vals;
        radix_sort_pairs<uint64_t>(A, &kk, &vv, B.keys_alt, B.vals_alt, total, 0, 32 + bits_for(nl), st);
        k_seg_large_scatter<<<grid_for(nl, 1, 4096), BLOCK, 0, st>>>(off, B.large, nl, data, B.pos, kk, uniq, usize);
        HGP_LAUNCH_CHECK();
    }
}

}  // namespace hgp
