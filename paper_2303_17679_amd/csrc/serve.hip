// Many hypergraphs at once: a partition server with continuous admission
// (hgp_server_*) and the batch call built on it (hgp_partition_batch).
//
// Host-side runtime only; every request runs the same multilevel driver as
// hgp_partition, so each result is bit-identical to a call on its own.
//  - lanes: one worker thread and one HIP stream per lane (default priority);
//    work of different lanes overlaps on the device;
//  - memory: the caller's pool is carved by a first-fit allocator with
//    coalescing; a request needs hgp_workspace_bytes(HGP_OP_PARTITION) of it;
//  - admission: arrival order, except that a request whose workspace does not
//    fit may be passed by later ones; after AGING passes it waits alone at
//    the head until it fits, so no request starves.
#include "hgp.h"
#include "timing.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint32_t AGING = 64;
constexpr uint32_t MAX_LANES = 64;
constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Pool {
public:
    explicit Pool(size_t size) { if (size) free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Request {
    hgp_hg h;
    hgp_params prm;
    uint32_t *part;
    int64_t *objective;
    size_t need = 0, off = 0;
    hipEvent_t ready = nullptr;  // inputs produced on the submitter's stream
    uint32_t passed = 0;         // times a later request was admitted first
    bool done = false;
    hgp_status status = HGP_OK;
    uint32_t levels = 0;
    Clock::time_point t_submit, t_start, t_end;
};

}  // namespace

struct hgp_server {
    int dev = 0;
    char *base = nullptr;
    size_t capacity = 0;
    Pool pool{0};
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    uint32_t running = 0;
    bool stop = false;

    // Next admissible request (caller holds mu): arrival order, first whose
    // workspace fits; a request passed AGING times blocks the others.
    bool take(uint64_t *ticket) {
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            Request &r = reqs[queue[qi]];
            size_t off;
            if (pool.alloc(r.need, &off)) {
                r.off = off;
                *ticket = queue[qi];
                for (size_t j = 0; j < qi; ++j) ++reqs[queue[j]].passed;
                queue.erase(queue.begin() + (long)qi);
                return true;
            }
            if (r.passed >= AGING) return false;
        }
        return false;
    }

    void work(uint32_t lane) {
        hipSetDevice(dev);
        hgp::blocking_waits = true;
        hipStream_t st = streams[lane];
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            uint64_t t = 0;
            cv_work.wait(lk, [&] { return stop || take(&t); });
            if (t == 0) return;  // stop with nothing admissible left
            Request &r = reqs[t];
            ++running;
            r.t_start = Clock::now();
            const hgp_hg h = r.h;
            const hgp_params prm = r.prm;
            uint32_t *part = r.part;
            int64_t *obj = r.objective;
            void *ws = base + r.off;
            const size_t need = r.need;
            hipEvent_t ready = r.ready;
            lk.unlock();
            hgp_status s = HGP_OK;
            if (ready && hipStreamWaitEvent(st, ready, 0) != hipSuccess) s = HGP_E_DEVICE;
            uint32_t lv = 0;
            if (s == HGP_OK) s = hgp_partition(&h, &prm, part, obj, &lv, ws, need, st);
            lk.lock();
            Request &q = reqs[t];
            q.t_end = Clock::now();
            q.status = s;
            q.levels = lv;
            q.done = true;
            if (q.ready) { hipEventDestroy(q.ready); q.ready = nullptr; }
            pool.release(q.off, q.need);
            --running;
            cv_done.notify_all();
            cv_work.notify_all();  // freed memory may admit waiting requests
        }
    }
};

extern "C" {

hgp_status hgp_server_create(uint32_t lanes, void *pool, size_t pool_bytes, hgp_server **out) {
    if (!out || !pool || lanes == 0 || lanes > MAX_LANES) return HGP_E_INVALID;
    if (((uintptr_t)pool & (ALIGN - 1)) != 0) return HGP_E_INVALID;
    if (hgp::timing().mask) return HGP_E_INVALID;  // measurement is single-stream only
    hgp_server *S = new hgp_server;
    if (hipGetDevice(&S->dev) != hipSuccess) { delete S; return HGP_E_DEVICE; }
    S->base = (char *)pool;
    S->capacity = pool_bytes & ~(ALIGN - 1);
    S->pool = Pool(S->capacity);
    S->streams.resize(lanes, nullptr);
    for (uint32_t l = 0; l < lanes; ++l) {
        if (hipStreamCreateWithFlags(&S->streams[l], hipStreamNonBlocking) != hipSuccess) {
            for (uint32_t q = 0; q < l; ++q) hipStreamDestroy(S->streams[q]);
            delete S;
            return HGP_E_DEVICE;
        }
    }
    for (uint32_t l = 0; l < lanes; ++l) S->workers.emplace_back([S, l] { S->work(l); });
    *out = S;
    return HGP_OK;
}

hgp_status hgp_server_submit(hgp_server *S, const hgp_hg *h, const hgp_params *prm, uint32_t *part,
                             int64_t *objective, void *stream, uint64_t *ticket) {
    if (!S || !h || !prm || !part || !objective || !ticket) return HGP_E_INVALID;
    size_t need = 0;
    hgp_status s = hgp_workspace_bytes(HGP_OP_PARTITION, h->n, h->m, h->p, prm, &need);
    if (s != HGP_OK) return s;
    if (h->n == 0 || !h->pin_off || !h->inc_off || !h->vwgt) return HGP_E_INVALID;
    Request r;
    r.h = *h;
    r.prm = *prm;
    r.part = part;
    r.objective = objective;
    r.need = align_up(need);
    r.t_submit = Clock::now();
    if (r.need > S->capacity) return HGP_E_WORKSPACE;  // could never be admitted
    if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess) return HGP_E_DEVICE;
    if (hipEventRecord(r.ready, (hipStream_t)stream) != hipSuccess) {
        hipEventDestroy(r.ready);
        return HGP_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        hipEventDestroy(r.ready);
        return HGP_E_INVALID;
    }
    const uint64_t t = S->next_ticket++;
    S->reqs.emplace(t, r);
    S->queue.push_back(t);
    *ticket = t;
    S->cv_work.notify_one();
    return HGP_OK;
}

hgp_status hgp_server_wait(hgp_server *S, uint64_t ticket, uint32_t *levels_out, double *latency_ms,
                           double *queue_ms) {
    if (!S) return HGP_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return HGP_E_INVALID;
    S->cv_done.wait(lk, [&] { return S->reqs[ticket].done; });
    Request r = S->reqs[ticket];
    S->reqs.erase(ticket);
    if (levels_out) *levels_out = r.levels;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_end - r.t_submit).count();
    if (queue_ms) *queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count();
    return r.status;
}

hgp_status hgp_server_destroy(hgp_server *S) {
    if (!S) return HGP_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (uint64_t t : S->queue) {  // never admitted: completed as cancelled
            Request &r = S->reqs[t];
            r.done = true;
            r.status = HGP_E_INVALID;
            r.t_start = r.t_end = Clock::now();
        }
        S->queue.clear();
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    for (auto &w : S->workers) w.join();
    for (auto &kv : S->reqs)
        if (kv.second.ready) hipEventDestroy(kv.second.ready);
    for (hipStream_t st : S->streams) hipStreamDestroy(st);
    delete S;
    return HGP_OK;
}

hgp_status hgp_batch_workspace_bytes(const hgp_hg *hs, const hgp_params *ps, uint32_t count, uint32_t lanes,
                                     size_t *out) {
    if (!out || (count && (!hs || !ps)) || lanes == 0 || lanes > MAX_LANES) return HGP_E_INVALID;
    size_t mx = 0;
    for (uint32_t i = 0; i < count; ++i) {
        size_t need = 0;
        hgp_status s = hgp_workspace_bytes(HGP_OP_PARTITION, hs[i].n, hs[i].m, hs[i].p, &ps[i], &need);
        if (s != HGP_OK) return s;
        mx = std::max(mx, align_up(need));
    }
    *out = mx * std::min<size_t>(lanes, std::max<uint32_t>(count, 1));
    return HGP_OK;
}

hgp_status hgp_partition_batch(const hgp_hg *hs, const hgp_params *ps, uint32_t count, uint32_t lanes,
                               uint32_t *const *parts, int64_t *objectives, uint32_t *levels_out, void *ws,
                               size_t ws_bytes, void *stream) {
    if ((count && (!hs || !ps || !parts || !objectives)) || !ws || lanes == 0 || lanes > MAX_LANES)
        return HGP_E_INVALID;
    if (count == 0) return HGP_OK;
    size_t need = 0;
    hgp_status s = hgp_batch_workspace_bytes(hs, ps, count, 1, &need);
    if (s != HGP_OK) return s;
    if (need > ws_bytes) return HGP_E_WORKSPACE;
    hgp_server *S = nullptr;
    s = hgp_server_create(std::min(lanes, count), ws, ws_bytes, &S);
    if (s != HGP_OK) return s;
    // largest first, so that the last requests to finish are small ones
    std::vector<uint32_t> order(count);
    for (uint32_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return hs[a].p > hs[b].p; });
    std::vector<uint64_t> tickets(count, 0);
    hgp_status first = HGP_OK;
    for (uint32_t q = 0; q < count && first == HGP_OK; ++q) {
        const uint32_t i = order[q];
        first = hgp_server_submit(S, &hs[i], &ps[i], parts[i], objectives + i, stream, &tickets[i]);
    }
    for (uint32_t i = 0; i < count; ++i) {
        if (!tickets[i]) continue;
        uint32_t lv = 0;
        hgp_status r = hgp_server_wait(S, tickets[i], &lv, nullptr, nullptr);
        if (levels_out) levels_out[i] = lv;
        if (r != HGP_OK && first == HGP_OK) first = r;
    }
    hgp_server_destroy(S);
    return first;
}

}  // extern "C"
