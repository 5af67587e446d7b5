// Subhypergraph extraction for the recursive-bipartitioning initial partition
// (paper Sec. 5; the subhypergraph H[V'] of Sec. 2).  V' = the vertices on
// one side of a bisection, renumbered in ascending ID; every net with a pin
// in V' is kept, restricted to those pins, in ascending net ID with its
// weight (single-pin nets included, as the definition has them).  Every net
// of a vertex of V' is kept, so a vertex's incidence list is its old list
// with the nets renumbered: no sort is needed.
#include "kernels.h"
#include "prims.h"

namespace hgp {

namespace {

constexpr uint32_t SUB_WIDE = 32;  // nets / lists longer than this: a wave each

// Vertices of the side, numbered by a scan of their flags.
struct SideFlag {
    const uint32_t *part;
    uint32_t side;
    __device__ uint32_t operator()(size_t v) const { return part[v] == side ? 1u : 0u; }
};
struct SideStore {
    const uint32_t *inc_off;
    const int32_t *vwgt;
    uint32_t *nid, *vmap, *deg;
    int32_t *vw;
    __device__ void operator()(size_t v, uint32_t excl, uint32_t f) const {
        if (f) {
            nid[v] = excl;
            vmap[excl] = (uint32_t)v;
            vw[excl] = vwgt[v];
            deg[excl] = inc_off[v + 1] - inc_off[v];
        } else {
            nid[v] = NONE;
        }
    }
};

// Pins of every net on the side (a thread per net, a wave per longer net).
__global__ __launch_bounds__(BLOCK) void k_sub_count(const uint32_t *pin_off, const uint32_t *pins, uint32_t m,
                                                     const uint32_t *nid, uint32_t *cnt) {
    for (uint32_t e0 = blockIdx.x * BLOCK; e0 < m; e0 += gridDim.x * BLOCK) {
        const uint32_t e = e0 + threadIdx.x;
        uint32_t b = 0, sz = 0;
        if (e < m) {
            b = pin_off[e];
            sz = pin_off[e + 1] - b;
        }
        const bool wide = sz > SUB_WIDE;
        if (e < m && !wide) {
            uint32_t c = 0;
            for (uint32_t q = b; q < b + sz; ++q) c += nid[pins[q]] != NONE;
            cnt[e] = c;
        }
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t he = __shfl(e, h, WAVE), hb = __shfl(b, h, WAVE), hs = __shfl(sz, h, WAVE);
            uint32_t c = 0;
            for (uint32_t q = hb + __lane_id(); q < hb + hs; q += WAVE) c += nid[pins[q]] != NONE;
            c = wave_sum(c);
            if ((int)__lane_id() == h) cnt[he] = c;
        }
    }
}

// Kept nets numbered by a scan of (1 << 32 | pins on the side).
struct NetPack {
    const uint32_t *cnt;
    __device__ uint64_t operator()(size_t e) const { return cnt[e] ? ((1ull << 32) | cnt[e]) : 0ull; }
};
struct NetStore {
    const int32_t *nwgt;
    uint32_t *nrank, *pin_off_s;
    int32_t *nwgt_s;
    uint32_t cap_m;
    __device__ void operator()(size_t e, uint64_t excl, uint64_t v) const {
        const uint32_t r = (uint32_t)(excl >> 32);
        nrank[e] = v ? r : NONE;
        if (v && r < cap_m) {
            pin_off_s[r] = (uint32_t)excl;
            nwgt_s[r] = nwgt[e];
        }
    }
};

// The kept pins of every kept net, in order (a wave compacts a long net with
// ballots, 64 pins at a time).
__global__ __launch_bounds__(BLOCK) void k_sub_pins(const uint32_t *pin_off, const uint32_t *pins, uint32_t m,
                                                    const uint32_t *nid, const uint32_t *nrank,
                                                    const uint32_t *pin_off_s, uint32_t *pins_s) {
    for (uint32_t e0 = blockIdx.x * BLOCK; e0 < m; e0 += gridDim.x * BLOCK) {
        const uint32_t e = e0 + threadIdx.x;
        uint32_t b = 0, sz = 0, o = 0;
        bool kept = false;
        if (e < m) {
            kept = nrank[e] != NONE;
            b = pin_off[e];
            sz = pin_off[e + 1] - b;
            if (kept) o = pin_off_s[nrank[e]];
        }
        const bool wide = kept && sz > SUB_WIDE;
        if (kept && !wide)
            for (uint32_t q = b; q < b + sz; ++q) {
                const uint32_t x = nid[pins[q]];
                if (x != NONE) pins_s[o++] = x;
            }
        uint64_t wm = __ballot(wide);
        while (wm) {
            const int h = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint32_t hb = __shfl(b, h, WAVE), hs = __shfl(sz, h, WAVE);
            uint32_t ho = __shfl(o, h, WAVE);
            for (uint32_t q0 = hb; q0 < hb + hs; q0 += WAVE) {
                const uint32_t q = q0 + __lane_id();
                const uint32_t x = q < hb + hs ? nid[pins[q]] : NONE;
                const uint64_t keep = __ballot(x != NONE);
                if (x != NONE) pins_s[ho + (uint32_t)__popcll(keep & lanemask_lt())] = x;
                ho += (uint32_t)__popcll(keep);
            }
        }
    }
}

// Incidence lists: vertex i's nets renumbered, a wave per vertex (the lanes
// stride over its list; coarse vertices have hundreds of nets).
__global__ __launch_bounds__(BLOCK) void k_sub_inc(const uint32_t *inc_off, const uint32_t *inc, uint32_t n2,
                                                   const uint32_t *vmap, const uint32_t *nrank,
                                                   const uint32_t *inc_off_s, uint32_t *inc_s) {
    const uint32_t wpb = BLOCK / WAVE;
    for (uint32_t i = blockIdx.x * wpb + threadIdx.x / WAVE; i < n2; i += gridDim.x * wpb) {
        const uint32_t v = vmap[i], j0 = inc_off[v], j1 = inc_off[v + 1], o = inc_off_s[i];
        for (uint32_t j = j0 + __lane_id(); j < j1; j += WAVE) inc_s[o + (j - j0)] = nrank[inc[j]];
    }
}

__global__ void k_set_word(uint32_t *p, const uint32_t *from) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = *from;
}

__global__ void k_set_value(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_gather_map(const uint32_t *outer, const uint32_t *inner, uint32_t n, uint32_t *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[i] = outer[inner[i]];
}

__global__ void k_assign_block(const uint32_t *vmap, uint32_t n, uint32_t b, uint32_t *part) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) part[vmap[i]] = b;
}

}  // namespace

void subhypergraph(const hgp_hg &h, const uint32_t *part, uint32_t side, const hgp_hg_out &out, uint32_t *vmap,
                   uint32_t *dims_host, Arena &A, hipStream_t st) {
    const uint32_t n = h.n, m = h.m;
    size_t mk = A.mark();
    uint32_t *nid = A.alloc<uint32_t>(n);
    uint32_t *deg = A.alloc<uint32_t>(n);
    uint32_t *cnt = A.alloc<uint32_t>(m ? m : 1);
    uint32_t *nrank = A.alloc<uint32_t>(m ? m : 1);
    uint32_t *d_n2 = A.alloc<uint32_t>(4);
    uint64_t *d_mp = A.alloc<uint64_t>(2);
    if (A.measure) { A.release(mk); return; }
    scan_apply<uint32_t>(A, n, SideFlag{part, side}, SideStore{h.inc_off, h.vwgt, nid, vmap, deg, out.vwgt}, d_n2,
                         st);
    if (m) {
        k_sub_count<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, m, nid, cnt);
        HGP_LAUNCH_CHECK();
    }
    scan_apply<uint64_t>(A, m, NetPack{cnt}, NetStore{h.nwgt, nrank, out.pin_off, out.nwgt, out.cap_m}, d_mp, st);
    uint32_t n2 = 0;
    uint64_t mp = 0;
    read_back({{&n2, d_n2, sizeof(uint32_t)}, {&mp, d_mp, sizeof(uint64_t)}}, st);
    const uint32_t m2 = (uint32_t)(mp >> 32), p2 = (uint32_t)mp;
    HGP_REQUIRE(n2 <= out.cap_n && m2 <= out.cap_m && p2 <= out.cap_p, HGP_E_INVALID);
    k_set_value<<<1, 64, 0, st>>>(out.pin_off + m2, p2);
    HGP_LAUNCH_CHECK();
    if (m) {
        k_sub_pins<<<grid_for(m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, m, nid, nrank, out.pin_off,
                                                                      out.pins);
        HGP_LAUNCH_CHECK();
    }
    // incidence offsets: the exclusive prefix of the side's degrees
    scan_apply<uint32_t>(A, n2, LoadArr<uint32_t>{deg}, StoreExcl<uint32_t>{out.inc_off}, d_n2 + 1, st);
    k_set_word<<<1, 64, 0, st>>>(out.inc_off + n2, d_n2 + 1);
    HGP_LAUNCH_CHECK();
    if (n2) {
        k_sub_inc<<<grid_for((size_t)n2 * WAVE, BLOCK, 4 * FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, h.inc, n2, vmap,
                                                                                       nrank, out.inc_off, out.inc);
        HGP_LAUNCH_CHECK();
    }
    dims_host[0] = n2;
    dims_host[1] = m2;
    dims_host[2] = p2;
    A.release(mk);
}

void gather_map(const uint32_t *outer, const uint32_t *inner, uint32_t n, uint32_t *out, hipStream_t st) {
    if (!n) return;
    k_gather_map<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(outer, inner, n, out);
    HGP_LAUNCH_CHECK();
}

void iota_u32(uint32_t *p, uint32_t n, hipStream_t st) {
    if (!n) return;
    k_iota<uint32_t><<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(p, n);
    HGP_LAUNCH_CHECK();
}

void assign_block(const uint32_t *vmap, uint32_t n, uint32_t b, uint32_t *part, hipStream_t st) {
    if (!n) return;
    k_assign_block<<<grid_for(n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(vmap, n, b, part);
    HGP_LAUNCH_CHECK();
}

}  // namespace hgp
