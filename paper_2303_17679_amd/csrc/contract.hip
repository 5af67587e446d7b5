// Contraction of a clustering (paper Sec. 4.2).
//
// Steps, each a data-parallel kernel over vertices, pins or nets:
//  1. coarse IDs: exclusive scan of the representative flags (ascending
//     representative ID), cid[v] = rank[rep[v]]; cluster weights by integer
//     atomics;
//  2. every pin replaced by its coarse ID, then each net sorted ascending and
//     de-duplicated (segmented sort, three tiers by net size);
//  3. nets of fewer than two pins are dropped; identical nets are found by
//     sorting the remaining nets by a 32-bit hash of their pin list (stable,
//     so equal hashes stay in ascending net ID) and comparing pin lists
//     exactly inside runs of equal hash: the kept net is the first identical
//     one in its run, i.e. the smallest net ID, and receives the summed
//     weight.  The hash only groups; it never decides identity (the paper's
//     fingerprint sum of squares plays the same filtering role);
//  4. kept nets numbered by one packed (count, pins) exclusive scan in
//     ascending fine ID; pins copied;
//  5. incidence arrays: degree count, scan, scatter, per-vertex sort.
#include "segsort.h"
#include "kernels.h"

namespace hgp {

struct IsRep {
    const uint32_t *rep;
    __device__ uint32_t operator()(size_t i) const { return rep[i] == (uint32_t)i ? 1u : 0u; }
};
struct StoreRank {
    uint32_t *rank;
    __device__ void operator()(size_t i, uint32_t excl, uint32_t) const { rank[i] = excl; }
};

// Coarse IDs and weights; the weights only below cap (the host rejects a
// coarse level above the caller's capacity once the count is read back).
__global__ void k_cid(const uint32_t *rep, const uint32_t *rank, uint32_t n, const int32_t *vwgt, uint32_t *cid,
                      int32_t *cvwgt, uint32_t cap) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        uint32_t c = rank[rep[v]];
        cid[v] = c;
        if (c < cap) atomicAdd(&cvwgt[c], vwgt[v]);
    }
}

__global__ void k_map_pins(const uint32_t *pins, size_t p, const uint32_t *cid, uint32_t *out) {
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < p; q += (size_t)gridDim.x * blockDim.x)
        out[q] = cid[pins[q]];
}

// Hash of a sorted distinct pin list (only groups candidates for identity).
__device__ inline uint64_t pin_hash_term(uint32_t x) { return mix64((uint64_t)x + 0x9E3779B97F4A7C15ULL); }

__global__ void k_net_hash_small(const uint32_t *off, uint32_t m, const uint32_t *tmp, const uint32_t *usize,
                                 uint32_t *hkey, uint8_t *valid) {
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
        uint32_t b = off[e], len = off[e + 1] - b;
        if (len > SEG_WAVE) continue;  // done by the block kernel
        uint32_t sz = usize[e];
        uint64_t h = 0;
        for (uint32_t i = 0; i < sz; ++i) h += pin_hash_term(tmp[b + i]);
        h = mix64(h ^ ((uint64_t)sz << 40));
        hkey[e] = (uint32_t)(h >> 32);
        valid[e] = sz >= 2;
    }
}

__global__ __launch_bounds__(BLOCK) void k_net_hash_block(const uint32_t *off, const uint32_t *list, uint32_t count,
                                                          const uint32_t *tmp, const uint32_t *usize, uint32_t *hkey,
                                                          uint8_t *valid) {
    __shared__ uint64_t red[BLOCK / WAVE];
    for (uint32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        uint32_t e = list[idx];
        uint32_t b = off[e], sz = usize[e];
        uint64_t h = 0;
        for (uint32_t i = threadIdx.x; i < sz; i += BLOCK) h += pin_hash_term(tmp[b + i]);
        h = wave_sum(h);
        if (__lane_id() == 0) red[threadIdx.x / WAVE] = h;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t t = 0;
            for (int q = 0; q < BLOCK / WAVE; ++q) t += red[q];
            t = mix64(t ^ ((uint64_t)sz << 40));
            hkey[e] = (uint32_t)(t >> 32);
            valid[e] = sz >= 2;
        }
        __syncthreads();
    }
}

struct IsValid {
    const uint8_t *valid;
    __device__ uint32_t operator()(size_t i) const { return valid[i]; }
};
struct GatherValid {
    const uint8_t *valid;
    const uint32_t *hkey;
    uint32_t *keys;
    uint32_t *vals;
    __device__ void operator()(size_t i, uint32_t excl, uint32_t v) const {
        if (v) {
            keys[excl] = hkey[i];
            vals[excl] = (uint32_t)i;
        }
    }
};

// Representative of every valid net: the first net, in the order the nets
// are sorted by the upper bits of their hash (stably, so by net within equal
// bits; see hash_sort_bits), with an identical pin list -- the smallest net ID
// among identical nets.  The run of equal sorted bits is found by stepping
// back over a few neighbours (runs are short), else by binary search.
// wsum[r] receives the weights of the nets r represents besides itself.
// repnet (NONE on entry) is written only for the nets that are merged into
// another one, so a net with no copy costs no scattered store.
// More nets than 2^24 (runs of about m / 2^24 nets per bucket) sort by all
// 32 bits, so that a net is compared only with the nets of equal hash.
constexpr int HASH_SORT_BITS = 24;
constexpr uint32_t HASH_FULL_SORT = 1u << 24;
__host__ __device__ inline int hash_sort_bits(uint32_t m) { return m > HASH_FULL_SORT ? 32 : HASH_SORT_BITS; }
__global__ void k_identical(const uint32_t *keys, const uint32_t *vals, const uint32_t *nv_dev, const uint32_t *off,
                            const uint32_t *tmp, const uint32_t *usize, const int32_t *nwgt, uint32_t *repnet,
                            int32_t *wsum, int SH) {
    const uint32_t nv = *nv_dev;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
        const uint32_t key = keys[i], top = key >> SH;
        uint32_t lo = i;
        int steps = 0;
        while (lo > 0 && steps < 4 && (keys[lo - 1] >> SH) == top) { --lo; ++steps; }
        if (lo > 0 && (keys[lo - 1] >> SH) == top) {  // a long run
            uint32_t a = 0, b = lo;
            while (a < b) {
                const uint32_t mid = (a + b) >> 1;
                if ((keys[mid] >> SH) < top) a = mid + 1; else b = mid;
            }
            lo = a;
        }
        const uint32_t e = vals[i];
        uint32_t r = e;
        if (lo < i) {
            const uint32_t sz = usize[e];
            const uint32_t *pe = tmp + off[e];
            for (uint32_t j = lo; j < i; ++j) {
                if (keys[j] != key) continue;
                const uint32_t f = vals[j];
                if (usize[f] != sz) continue;
                const uint32_t *pf = tmp + off[f];
                bool same = true;
                for (uint32_t q = 0; q < sz && same; ++q) same = pe[q] == pf[q];
                if (same) { r = f; break; }
            }
            if (r != e) {
                atomicAdd(&wsum[r], nwgt[e]);
                repnet[e] = r;
            }
        }
    }
}

// Packed (count << 32 | pins) of kept nets.
struct KeptPack {
    const uint8_t *valid;
    const uint32_t *repnet, *usize;
    __device__ uint64_t operator()(size_t e) const {
        return (valid[e] && repnet[e] == NONE) ? ((1ull << 32) | usize[e]) : 0ull;
    }
};
struct StoreKept {
    uint32_t *newid, *newoff, *cpin_off;
    int32_t *cnwgt;
    const int32_t *nwgt, *wsum;
    uint32_t cap_m;  // coarse arrays written below it only (the host checks mc <= cap_m)
    __device__ void operator()(size_t e, uint64_t excl, uint64_t v) const {
        if (v) {
            uint32_t id = (uint32_t)(excl >> 32);
            newid[e] = id;
            newoff[e] = (uint32_t)excl;
            if (id < cap_m) {
                cpin_off[id] = (uint32_t)excl;
                cnwgt[id] = nwgt[e] + wsum[e];
            }
        } else {
            newid[e] = NONE;
        }
    }
};

// Pins of the kept nets into the coarse pin array, and (pin, net) pairs in
// net order for the transpose: sorting them stably by pin gives every coarse
// vertex its incident nets in increasing order.
// A wave takes WAVE consecutive nets (a net per lane) and copies their kept
// pins together, WAVE pins per step: a wave prefix of the sizes numbers the
// pins, and each lane finds the net of its pin by a binary search over the
// lanes' prefixes.  Consecutive nets have consecutive pin ranges on both
// sides, so the loads and stores of a step are nearly contiguous.
__global__ void k_copy_pins_small(const uint32_t *off, uint32_t m, const uint32_t *tmp, const uint32_t *usize,
                                  const uint32_t *newid, const uint32_t *newoff, uint32_t *cpins, uint32_t *tkey,
                                  uint32_t *tnet) {
    const uint32_t lane = __lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, nw = gridDim.x * blockDim.x / WAVE;
    for (uint32_t run = wid * WAVE; run < m; run += nw * WAVE) {  // uniform per wave
        const uint32_t e = run + lane;
        uint32_t id = NONE, b = 0, sz = 0, o = 0;
        if (e < m) {
            id = newid[e];
            if (id != NONE) {
                b = off[e];
                if (off[e + 1] - b <= SEG_WAVE) {  // longer nets: the block kernel
                    sz = usize[e];
                    o = newoff[e];
                }
            }
        }
        uint32_t x = sz;  // inclusive prefix over the lanes
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const uint32_t t = __shfl_up(x, d, WAVE);
            if (lane >= (uint32_t)d) x += t;
        }
        const uint32_t total = __shfl(x, WAVE - 1, WAVE), excl = x - sz;
        for (uint32_t q0 = 0; q0 < total; q0 += WAVE) {
            const uint32_t q = q0 + lane;
            uint32_t j = 0;  // the last lane whose prefix is <= q: its net holds pin q
#pragma unroll
            for (int step = WAVE / 2; step >= 1; step >>= 1) {
                const uint32_t c = j + (uint32_t)step;
                if (__shfl(excl, (int)c, WAVE) <= q) j = c;
            }
            const uint32_t bj = __shfl(b, (int)j, WAVE), oj = __shfl(o, (int)j, WAVE);
            const uint32_t idj = __shfl(id, (int)j, WAVE), ej = __shfl(excl, (int)j, WAVE);
            if (q < total) {
                const uint32_t i = q - ej, v = tmp[bj + i];
                cpins[oj + i] = v;
                tkey[oj + i] = v;
                tnet[oj + i] = idj;
            }
        }
    }
}

__global__ void k_copy_pins_block(const uint32_t *off, const uint32_t *list, uint32_t count, const uint32_t *tmp,
                                  const uint32_t *usize, const uint32_t *newid, const uint32_t *newoff,
                                  uint32_t *cpins, uint32_t *tkey, uint32_t *tnet) {
    for (uint32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        uint32_t e = list[idx];
        const uint32_t id = newid[e];
        if (id == NONE) continue;
        uint32_t b = off[e], sz = usize[e], o = newoff[e];
        for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) {
            uint32_t v = tmp[b + i];
            cpins[o + i] = v;
            tkey[o + i] = v;
            tnet[o + i] = id;
        }
    }
}

// Incidence offsets from the pins sorted by vertex: inc_off[v] is the first
// position whose vertex is >= v (every v in [0, nc] is written once).
__global__ void k_inc_offsets(const uint32_t *skey, uint32_t pc, uint32_t nc, uint32_t *inc_off) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= pc; i += gridDim.x * blockDim.x) {
        const uint32_t lo = i == 0 ? 0u : skey[i - 1] + 1;  // first vertex not yet started
        const uint32_t hi = i == pc ? nc : skey[i];         // last vertex that starts here
        for (uint32_t v = lo; v <= hi; ++v) inc_off[v] = i;
    }
}

struct ContractBufs {
    uint32_t *rank, *tmp, *usize, *hkey, *repnet, *newid, *newoff, *scal;
    int32_t *wsum;
    uint8_t *valid;
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
    uint32_t *tkey, *tkey_alt, *tnet;  // transpose: (pin, net) pairs and the sort's second buffer
    SegSortBufs ss_net;
};

static void plan(Arena &A, uint32_t n, uint32_t m, uint32_t p, ContractBufs &B) {
    B.rank = A.alloc<uint32_t>(n);
    B.tmp = A.alloc<uint32_t>(p);
    B.usize = A.alloc<uint32_t>(m);
    B.hkey = A.alloc<uint32_t>(m);
    B.repnet = A.alloc<uint32_t>(m);
    B.newid = A.alloc<uint32_t>(m);
    B.newoff = A.alloc<uint32_t>(m);
    B.scal = A.alloc<uint32_t>(8);
    B.wsum = A.alloc<int32_t>(m);
    B.valid = A.alloc<uint8_t>(m);
    B.keys = A.alloc<uint64_t>(m);
    B.keys_alt = A.alloc<uint64_t>(m);
    B.vals = A.alloc<uint32_t>(m);
    B.vals_alt = A.alloc<uint32_t>(m);
    B.tkey = A.alloc<uint32_t>(p);
    B.tkey_alt = A.alloc<uint32_t>(p);
    B.tnet = A.alloc<uint32_t>(p);
    segsort_plan(A, m, p, B.ss_net);
    scan_reserve<uint32_t>(A, (size_t)n + 1);
    scan_reserve<uint64_t>(A, m);
    sort_reserve(A, p > m ? p : m);
}

size_t contract_workspace(uint32_t n, uint32_t m, uint32_t p) {
    Arena A(nullptr, 0);
    ContractBufs B;
    plan(A, n, m, p, B);
    return A.peak;
}

// Up to three device words from host values, as kernel arguments: a copy from
// pageable host memory would be a host round trip of its own.
__global__ void k_put_words3(uint32_t *p, uint32_t n, uint32_t a, uint32_t b, uint32_t c) {
    if (blockIdx.x == 0 && threadIdx.x < n) p[threadIdx.x] = threadIdx.x == 0 ? a : (threadIdx.x == 1 ? b : c);
}

void contract(const hgp_hg &h, const uint32_t *rep, uint32_t *cid, const hgp_hg_out &out, uint32_t *dims_host,
              Arena &A, hipStream_t st) {
    const uint32_t n = h.n, m = h.m, p = h.p;
    size_t mk = A.mark();
    ContractBufs B;
    plan(A, n, m, p, B);
    uint32_t *d_nc = B.scal + 0;
    uint64_t *d_tot = (uint64_t *)(B.scal + 2);
    uint32_t *d_nv = B.scal + 4;

    // 1. coarse vertex IDs and weights; the cluster count is read back at
    // the segmented sort's sync
    scan_apply<uint32_t>(A, n, IsRep{rep}, StoreRank{B.rank}, d_nc, st);
    uint32_t *mb = host_mailbox();
    HGP_CHECK_HIP(hipMemcpyAsync(mb, d_nc, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    const uint32_t vcap = std::min(out.cap_n, n);  // nc <= n
    if (vcap) HGP_CHECK_HIP(hipMemsetAsync(out.vwgt, 0, sizeof(int32_t) * vcap, st));
    if (n) {
        k_cid<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(rep, B.rank, n, h.vwgt, cid, out.vwgt, vcap);
        HGP_LAUNCH_CHECK();
    }

    // 2. remap pins, sort + de-duplicate every net
    if (p) {
        k_map_pins<<<grid_for(p, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pins, p, cid, B.tmp);
        HGP_LAUNCH_CHECK();
    }
    uint32_t cnt_ml[2];
    segmented_sort(A, B.ss_net, h.pin_off, m, B.tmp, true, B.usize, cnt_ml, st);  // syncs
    const uint32_t nc = mb[0];
    HGP_REQUIRE(nc <= out.cap_n, HGP_E_INVALID);

    // 3. hashes, drop single-pin nets, identical-net detection
    if (m) {
        k_net_hash_small<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, m, B.tmp, B.usize, B.hkey,
                                                                           B.valid);
        HGP_LAUNCH_CHECK();
    }
    if (cnt_ml[0]) {
        k_net_hash_block<<<grid_for(cnt_ml[0], 1, 4096), BLOCK, 0, st>>>(h.pin_off, B.ss_net.med, cnt_ml[0], B.tmp,
                                                                         B.usize, B.hkey, B.valid);
        HGP_LAUNCH_CHECK();
    }
    if (cnt_ml[1]) {
        k_net_hash_block<<<grid_for(cnt_ml[1], 1, 4096), BLOCK, 0, st>>>(h.pin_off, B.ss_net.large, cnt_ml[1], B.tmp,
                                                                         B.usize, B.hkey, B.valid);
        HGP_LAUNCH_CHECK();
    }
    // the nv kept nets' (hash, net) pairs: their count stays on the device,
    // the launches are sized for m
    scan_apply<uint32_t>(A, m, IsValid{B.valid}, GatherValid{B.valid, B.hkey, (uint32_t *)B.keys, B.vals}, d_nv, st);
    uint32_t *kk = (uint32_t *)B.keys;  // 32-bit hash keys in the 64-bit buffers
    uint32_t *vv = B.vals;
    const int sbits = hash_sort_bits(m);
    radix_sort_pairs<uint32_t>(A, &kk, &vv, (uint32_t *)B.keys_alt, B.vals_alt, m, 32 - sbits, 32, st,
                               d_nv);
    if (m) {
        HGP_CHECK_HIP(hipMemsetAsync(B.wsum, 0, sizeof(int32_t) * m, st));
        HGP_CHECK_HIP(hipMemsetAsync(B.repnet, 0xFF, sizeof(uint32_t) * m, st));
        k_identical<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(kk, vv, d_nv, h.pin_off, B.tmp, B.usize,
                                                                      h.nwgt, B.repnet, B.wsum, 32 - sbits);
        HGP_LAUNCH_CHECK();
    }

    // 4. number the kept nets, copy pins, count coarse degrees
    scan_apply<uint64_t>(A, m, KeptPack{B.valid, B.repnet, B.usize},
                         StoreKept{B.newid, B.newoff, out.pin_off, out.nwgt, h.nwgt, B.wsum, out.cap_m}, d_tot, st);
    uint64_t tot = 0;
    read_back(&tot, d_tot, sizeof(uint64_t), st);
    uint32_t mc = (uint32_t)(tot >> 32), pc = (uint32_t)tot;
    HGP_REQUIRE(mc <= out.cap_m && pc <= out.cap_p, HGP_E_INVALID);
    k_put_words3<<<1, 64, 0, st>>>(out.pin_off + mc, 1, pc, 0, 0);
    HGP_LAUNCH_CHECK();
    // the transpose's net ids start where the stable sort by vertex (8-bit
    // digits) leaves them: in out.inc after an even number of passes
    const int vbits = bits_for(nc ? nc - 1 : 0);
    const bool even = ((vbits + 7) / 8) % 2 == 0;
    uint32_t *tnet = even ? out.inc : B.tnet, *tnet_alt = even ? B.tnet : out.inc;
    if (m) {
        k_copy_pins_small<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, m, B.tmp, B.usize, B.newid,
                                                                            B.newoff, out.pins, B.tkey, tnet);
        HGP_LAUNCH_CHECK();
    }
    if (cnt_ml[0]) {
        k_copy_pins_block<<<grid_for(cnt_ml[0], 1, 4096), BLOCK, 0, st>>>(h.pin_off, B.ss_net.med, cnt_ml[0], B.tmp,
                                                                          B.usize, B.newid, B.newoff, out.pins,
                                                                          B.tkey, tnet);
        HGP_LAUNCH_CHECK();
    }
    if (cnt_ml[1]) {
        k_copy_pins_block<<<grid_for(cnt_ml[1], 1, 4096), BLOCK, 0, st>>>(h.pin_off, B.ss_net.large, cnt_ml[1], B.tmp,
                                                                          B.usize, B.newid, B.newoff, out.pins,
                                                                          B.tkey, tnet);
        HGP_LAUNCH_CHECK();
    }

    // 5. incidence: the (pin, net) pairs sorted stably by pin (nets of a
    // vertex in increasing order), offsets from the sorted pins
    uint32_t *tk = B.tkey, *tv = tnet;
    radix_sort_pairs<uint32_t>(A, &tk, &tv, B.tkey_alt, tnet_alt, pc, 0, vbits, st);
    HGP_REQUIRE(pc == 0 || tv == out.inc, HGP_E_INVALID);
    if (pc) {
        k_inc_offsets<<<grid_for((size_t)pc + 1, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(tk, pc, nc, out.inc_off);
        HGP_LAUNCH_CHECK();
    } else {
        HGP_CHECK_HIP(hipMemsetAsync(out.inc_off, 0, sizeof(uint32_t) * ((size_t)nc + 1), st));
    }
    uint32_t dims[3] = {nc, mc, pc};
    if (out.dims) {
        k_put_words3<<<1, 64, 0, st>>>(out.dims, 3, dims[0], dims[1], dims[2]);
        HGP_LAUNCH_CHECK();
    }
    stream_sync(st);
    if (dims_host) { dims_host[0] = nc; dims_host[1] = mc; dims_host[2] = pc; }
    A.release(mk);
}

}  // namespace hgp
