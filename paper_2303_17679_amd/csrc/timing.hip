// Per-kernel event timing and compulsory-byte accounting (measurement only).
#include "timing.h"
#include "kernels.h"

namespace hgp {

Timing &timing() {
    static Timing t;
    return t;
}

static hipEvent_t get_event() {
    Timing &T = timing();
    if (!T.pool.empty()) {
        hipEvent_t e = T.pool.back();
        T.pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HGP_CHECK_HIP(hipEventCreate(&e));
    return e;
}

TimedLaunch::TimedLaunch(int k, hipStream_t s) : kid(k), st(s) {
    if (timing().account && (timing().mask >> kid & 1u)) timing().acc_launches[kid] += 1;
    Timing &T = timing();
    if (!T.account && (T.mask >> kid & 1u) && T.seen[kid]++ % T.every == T.phase) {
        e0 = get_event();
        e1 = get_event();
        HGP_CHECK_HIP(hipEventRecord(e0, st));
    }
}

TimedLaunch::~TimedLaunch() {
    if (e0) {
        hipEventRecord(e1, st);
        timing().pending[kid].push_back({e0, e1});
        timing().launches[kid] += 1;
    }
}

}  // namespace hgp

using namespace hgp;

extern "C" {

hgp_status hgp_timing_scratch_bytes(uint32_t n_max, uint32_t m_max, size_t *out) {
    if (!out) return HGP_E_INVALID;
    size_t len = (size_t)(n_max > m_max ? n_max : m_max) + 1;
    *out = 256 + 3 * len * sizeof(uint32_t);
    return HGP_OK;
}

hgp_status hgp_timing_begin(uint32_t mask, int account, void *scratch, size_t scratch_bytes, uint32_t n_max,
                            uint32_t m_max) {
    Timing &T = timing();
    for (int k = 0; k < KID_COUNT; ++k) {
        for (auto &p : T.pending[k]) { T.pool.push_back(p.first); T.pool.push_back(p.second); }
        T.pending[k].clear();
        T.launches[k] = 0;
        T.acc_launches[k] = 0;
        T.acc_host[k] = 0;
        T.seen[k] = 0;
    }
    T.every = 1;
    T.phase = 0;
    T.mask = mask & ((1u << KID_COUNT) - 1u);
    T.account = false;
    T.acc_dev = nullptr;
    T.marks = nullptr;
    if (account) {
        size_t need = 0;
        hgp_timing_scratch_bytes(n_max, m_max, &need);
        if (!scratch || scratch_bytes < need) return HGP_E_WORKSPACE;
        T.account = true;
        T.acc_dev = (uint64_t *)scratch;
        T.marks = (uint32_t *)((char *)scratch + 256);
        T.marks_len = (size_t)(n_max > m_max ? n_max : m_max) + 1;
        T.stamp = 0;
        if (hipMemset(scratch, 0, need) != hipSuccess) return HGP_E_DEVICE;
    }
    return HGP_OK;
}

hgp_status hgp_timing_sample(uint32_t every, uint32_t phase) {
    if (every == 0 || phase >= every) return HGP_E_INVALID;
    Timing &T = timing();
    T.every = every;
    T.phase = phase;
    for (int k = 0; k < KID_COUNT; ++k) T.seen[k] = 0;
    return HGP_OK;
}

hgp_status hgp_timing_end(uint32_t count, double *total_ms, uint64_t *launches, double *bytes) {
    Timing &T = timing();
    if (hipDeviceSynchronize() != hipSuccess) return HGP_E_DEVICE;
    uint64_t acc[KID_COUNT] = {};
    if (T.account && T.acc_dev)
        if (hipMemcpy(acc, T.acc_dev, sizeof(acc), hipMemcpyDeviceToHost) != hipSuccess) return HGP_E_DEVICE;
    for (uint32_t k = 0; k < count && k < (uint32_t)KID_COUNT; ++k) {
        double ms = 0;
        for (auto &p : T.pending[k]) {
            float x = 0;
            if (hipEventElapsedTime(&x, p.first, p.second) != hipSuccess) return HGP_E_DEVICE;
            ms += x;
        }
        if (total_ms) total_ms[k] = ms;
        if (launches) launches[k] = T.launches[k] ? T.launches[k] : T.acc_launches[k];
        if (bytes) bytes[k] = (double)acc[k] + T.acc_host[k];
    }
    for (int k = 0; k < KID_COUNT; ++k) {
        for (auto &p : T.pending[k]) { T.pool.push_back(p.first); T.pool.push_back(p.second); }
        T.pending[k].clear();
        T.launches[k] = 0;
        T.acc_launches[k] = 0;
    }
    T.mask = 0;
    T.account = false;
    return HGP_OK;
}

}  // extern "C"
