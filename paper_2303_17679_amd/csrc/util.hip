// Reductions needed on the host (total weights) and input validation.
#include "prims.h"
#include "kernels.h"
#include <cstring>

namespace hgp {

__global__ __launch_bounds__(BLOCK) void k_sum_max(const int32_t *w, uint32_t n, int64_t *sum, int32_t *mx,
                                                   uint32_t *nonpos) {
    __shared__ int64_t rs[BLOCK / WAVE];
    __shared__ int32_t rm[BLOCK / WAVE];
    int64_t s = 0;
    int32_t m = 0;
    bool bad = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int32_t x = w[i];
        s += x;
        m = x > m ? x : m;
        bad |= x < 1;
    }
    s = wave_sum(s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int32_t t = __shfl_xor(m, o, 64);
        m = t > m ? t : m;
    }
    if (__lane_id() == 0) { rs[threadIdx.x / WAVE] = s; rm[threadIdx.x / WAVE] = m; }
    if (bad) atomicOr(nonpos, 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t ts = 0;
        int32_t tm = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) { ts += rs[q]; tm = rm[q] > tm ? rm[q] : tm; }
        atomic_add_i64(sum, ts);
        atomicMax(mx, tm);
    }
}

struct SumMax {
    int64_t sum;
    int32_t max;
    bool nonpos;
};

static SumMax sum_max(const int32_t *w, uint32_t n, Arena &A, hipStream_t st) {
    size_t mk = A.mark();
    char *buf = A.alloc<char>(64);
    SumMax r{0, 0, false};
    if (A.measure) { A.release(mk); return r; }
    HGP_CHECK_HIP(hipMemsetAsync(buf, 0, 64, st));
    if (n) {
        k_sum_max<<<grid_for(n, BLOCK * 8, REDUCE_BLOCKS), BLOCK, 0, st>>>(w, n, (int64_t *)buf, (int32_t *)(buf + 8),
                                                                  (uint32_t *)(buf + 12));
        HGP_LAUNCH_CHECK();
    }
    char host[16];
    read_back(host, buf, 16, st, false);
    r.sum = *(int64_t *)host;
    r.max = *(int32_t *)(host + 8);
    r.nonpos = *(uint32_t *)(host + 12) != 0;
    A.release(mk);
    return r;
}

int64_t total_weight(const int32_t *w, uint32_t n, Arena &A, hipStream_t st) { return sum_max(w, n, A, st).sum; }
int32_t max_vertex_weight(const int32_t *w, uint32_t n, Arena &A, hipStream_t st) { return sum_max(w, n, A, st).max; }

// ---------------------------------------------------------------------------
// Validation (bit 0: offsets, bit 1: ids/order, bit 2: transpose)
// ---------------------------------------------------------------------------
__global__ void k_check_offsets(const uint32_t *off, uint32_t cnt, uint32_t total, uint32_t *err) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= cnt; i += gridDim.x * blockDim.x) {
        uint32_t o = off[i];
        if (i == 0 && o != 0) atomicOr(err, 1u);
        if (i == cnt && o != total) atomicOr(err, 1u);
        if (i < cnt && off[i + 1] < o) atomicOr(err, 1u);
        if (o > total) atomicOr(err, 1u);
    }
}

// ids strictly ascending and < bound inside every segment
__global__ __launch_bounds__(BLOCK) void k_check_lists(const uint32_t *off, const uint32_t *data, uint32_t cnt,
                                                       uint32_t bound, uint32_t *err) {
    // every list strictly ascending and below `bound`; lists of more than 32
    // entries are checked by their whole wave
    for (uint32_t s0 = blockIdx.x * BLOCK; s0 < cnt; s0 += gridDim.x * BLOCK) {
        const uint32_t s = s0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (s < cnt) { j0 = off[s]; j1 = off[s + 1]; }
        const bool heavy = j1 - j0 > 32;
        if (!heavy) {
            uint32_t prev = 0;
            for (uint32_t j = j0; j < j1; ++j) {
                const uint32_t x = data[j];
                if (x >= bound || (j > j0 && x <= prev)) { atomicOr(err, 2u); break; }
                prev = x;
            }
        }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int h = __ffsll((long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t hj0 = __shfl(j0, h, 64), hj1 = __shfl(j1, h, 64);
            bool bad = false;
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) {
                const uint32_t x = data[j];
                bad |= x >= bound || (j > hj0 && x <= data[j - 1]);
            }
            if (__ballot(bad) && __lane_id() == 0) atomicOr(err, 2u);
        }
    }
}

// every pin (e, v) appears as e in v's incidence list (both sides hold p
// distinct pairs, so this makes the incidence the exact transpose)
__global__ __launch_bounds__(BLOCK) void k_check_transpose(const uint32_t *pin_off, const uint32_t *pins, uint32_t m,
                                                           const uint32_t *inc_off, const uint32_t *inc,
                                                           uint32_t *err) {
    // every pin (e, v) appears in v's incidence list (binary search); nets of
    // more than 32 pins are checked by their whole wave
    for (uint32_t e0 = blockIdx.x * BLOCK; e0 < m; e0 += gridDim.x * BLOCK) {
        const uint32_t e = e0 + threadIdx.x;
        uint32_t j0 = 0, j1 = 0;
        if (e < m) { j0 = pin_off[e]; j1 = pin_off[e + 1]; }
        const bool heavy = j1 - j0 > 32;
        auto found = [&](uint32_t net, uint32_t v) {
            uint32_t lo = inc_off[v], hi = inc_off[v + 1];
            const uint32_t end = hi;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (inc[mid] < net) lo = mid + 1; else hi = mid;
            }
            return lo < end && inc[lo] == net;
        };
        if (!heavy) {  // eight pins at a time, their binary searches in lock step
            bool ok = true;
            for (uint32_t j = j0; j < j1 && ok; j += 8) {
                uint32_t v[8], lo[8], hi[8], end[8];
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) v[q] = j + q < j1 ? pins[j + q] : NONE;
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) {
                    lo[q] = v[q] != NONE ? inc_off[v[q]] : 0u;
                    hi[q] = v[q] != NONE ? inc_off[v[q] + 1] : 0u;
                    end[q] = hi[q];
                }
                for (bool any = true; any;) {
                    any = false;
                    uint32_t x[8];
#pragma unroll
                    for (uint32_t q = 0; q < 8; ++q) x[q] = lo[q] < hi[q] ? inc[(lo[q] + hi[q]) >> 1] : 0u;
#pragma unroll
                    for (uint32_t q = 0; q < 8; ++q) {
                        if (lo[q] >= hi[q]) continue;
                        const uint32_t mid = (lo[q] + hi[q]) >> 1;
                        if (x[q] < e) lo[q] = mid + 1; else hi[q] = mid;
                        any = true;
                    }
                }
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q)
                    if (v[q] != NONE) ok = ok && lo[q] < end[q] && inc[lo[q]] == e;
            }
            if (!ok) atomicOr(err, 4u);
        }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int h = __ffsll((long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t he = __shfl(e, h, 64), hj0 = __shfl(j0, h, 64), hj1 = __shfl(j1, h, 64);
            bool bad = false;
            for (uint32_t j = hj0 + __lane_id(); j < hj1; j += WAVE) bad |= !found(he, pins[j]);
            if (__ballot(bad) && __lane_id() == 0) atomicOr(err, 4u);
        }
    }
}

size_t util_workspace(uint32_t, uint32_t) { return 4096; }

hgp_status validate(const hgp_hg &h, Arena &A, hipStream_t st) {
    size_t mk = A.mark();
    uint32_t *err = A.alloc<uint32_t>(4);
    if (A.measure) { A.release(mk); return HGP_OK; }
    uint32_t e = 0;
    HGP_CHECK_HIP(hipMemsetAsync(err, 0, 16, st));
    k_check_offsets<<<grid_for((size_t)h.m + 1, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.m, h.p, err);
    HGP_LAUNCH_CHECK();
    k_check_offsets<<<grid_for((size_t)h.n + 1, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, h.n, h.p, err);
    HGP_LAUNCH_CHECK();
    HGP_CHECK_HIP(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st));
    stream_sync(st);
    if (e) { A.release(mk); return HGP_E_INVALID; }
    if (h.m) {
        k_check_lists<<<grid_for(h.m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, h.m, h.n, err);
        HGP_LAUNCH_CHECK();
    }
    k_check_lists<<<grid_for(h.n, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.inc_off, h.inc, h.n, h.m, err);
    HGP_LAUNCH_CHECK();
    HGP_CHECK_HIP(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st));
    stream_sync(st);
    if (e) { A.release(mk); return HGP_E_INVALID; }
    if (h.m) {
        k_check_transpose<<<grid_for(h.m, BLOCK, FILL_BLOCKS), BLOCK, 0, st>>>(h.pin_off, h.pins, h.m, h.inc_off,
                                                                              h.inc, err);
        HGP_LAUNCH_CHECK();
    }
    HGP_CHECK_HIP(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st));
    stream_sync(st);
    A.release(mk);
    if (e) return HGP_E_INVALID;
    SumMax vw = sum_max(h.vwgt, h.n, A, st);
    SumMax nw = sum_max(h.nwgt, h.m, A, st);
    if (vw.nonpos || nw.nonpos) return HGP_E_INVALID;
    if (vw.sum >= (int64_t)1 << 31 || nw.sum >= (int64_t)1 << 31) return HGP_E_OVERFLOW;
    return HGP_OK;
}

namespace {
struct WaitEvent {
    hipEvent_t ev = nullptr;
    ~WaitEvent() {
        if (ev) hipEventDestroy(ev);
    }
};
}  // namespace

namespace {
struct PinnedWords {
    uint32_t *p = nullptr;
    ~PinnedWords() {
        if (p) hipHostFree(p);
    }
};
}  // namespace

uint32_t *host_mailbox() {
    thread_local PinnedWords w;
    if (!w.p) HGP_CHECK_HIP(hipHostMalloc((void **)&w.p, sizeof(uint32_t) * MAILBOX_WORDS, hipHostMallocDefault));
    return w.p;
}

void read_back(std::initializer_list<HostRead> reads, hipStream_t st, bool may_allocate) {
    thread_local PinnedWords stage;
    if (!stage.p && may_allocate)
        HGP_CHECK_HIP(hipHostMalloc((void **)&stage.p, STAGE_BYTES, hipHostMallocDefault));
    char *base = (char *)stage.p;
    const size_t cap = base ? STAGE_BYTES : 0;
    size_t used = 0;
    for (const HostRead &r : reads) {
        if (!r.bytes) continue;
        const size_t at = (used + 15) & ~(size_t)15;
        if (at + r.bytes <= cap) {
            HGP_CHECK_HIP(hipMemcpyAsync(base + at, r.src, r.bytes, hipMemcpyDeviceToHost, st));
            used = at + r.bytes;
        } else {
            HGP_CHECK_HIP(hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToHost, st));
        }
    }
    stream_sync(st);
    used = 0;
    for (const HostRead &r : reads) {
        if (!r.bytes) continue;
        const size_t at = (used + 15) & ~(size_t)15;
        if (at + r.bytes <= cap) {
            std::memcpy(r.dst, base + at, r.bytes);
            used = at + r.bytes;
        }
    }
}

void stream_sync(hipStream_t st) {
    if (!blocking_waits) {
        HGP_CHECK_HIP(hipStreamSynchronize(st));
        return;
    }
    thread_local WaitEvent w;
    if (!w.ev) HGP_CHECK_HIP(hipEventCreateWithFlags(&w.ev, hipEventBlockingSync | hipEventDisableTiming));
    HGP_CHECK_HIP(hipEventRecord(w.ev, st));
    HGP_CHECK_HIP(hipEventSynchronize(w.ev));
}

}  // namespace hgp
