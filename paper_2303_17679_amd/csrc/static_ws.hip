// Entry point that allocates nothing: label-propagation refinement with its
// scratch memory in a file-scope device array instead of a caller workspace.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  Each
// device that loads the library holds one array of HGP_STATIC_SCRATCH_BYTES
// until the process ends.  Every call on a device shares that device's
// array and finds the previous call's contents in it; the LP driver clears
// every counter, flag and stamp it reads at the start of the call, so no
// state carries over.  Calls that overlap on one device (two host threads, or
// two streams without ordering between them) race on the array.
#include "kernels.h"

#include <mutex>

using namespace hgp;

static __device__ __align__(256) unsigned char scratch[HGP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

// The array's device address on each device.  In host code `scratch` is a
// host-side stand-in, not a device address: it is only ever passed to
// hipGetSymbolAddress, with the device current, once per device.
struct ScratchTable {
    std::mutex mu;
    void *ptr[MAX_DEVICES] = {};
};

ScratchTable &table() {
    static ScratchTable t;
    return t;
}

hgp_status scratch_of_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return HGP_E_DEVICE;
    if (dev >= MAX_DEVICES) return HGP_E_UNSUPPORTED;
    ScratchTable &T = table();
    std::lock_guard<std::mutex> lk(T.mu);
    if (!T.ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HGP_E_DEVICE;
        T.ptr[dev] = p;
    }
    *out = T.ptr[dev];
    return HGP_OK;
}

}  // namespace

extern "C" {

hgp_status hgp_refine_lp_static(const hgp_hg *h, const hgp_params *prm, uint32_t level, uint32_t *part,
                                int64_t *objective, int64_t *block_wgt, void *stream) {
    if (!h || !prm || !part) return HGP_E_INVALID;
    size_t need = 0;
    hgp_status s = hgp_workspace_bytes(HGP_OP_REFINE, h->n, h->m, h->p, prm, &need);
    if (s != HGP_OK) return s;
    if (need > (size_t)HGP_STATIC_SCRATCH_BYTES) return HGP_E_WORKSPACE;  // nothing enqueued
    void *ws = nullptr;
    s = scratch_of_current_device(&ws);
    if (s != HGP_OK) return s;
    return hgp_refine_lp(h, prm, level, part, objective, block_wgt, ws, (size_t)HGP_STATIC_SCRATCH_BYTES, stream);
}

}  // extern "C"
