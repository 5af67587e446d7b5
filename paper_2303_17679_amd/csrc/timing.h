// Measurement support: per-kernel HIP-event timing on the launch stream and
// exact accounting of the compulsory (algorithmic) bytes of each launch.
// Host-side state only; nothing here runs unless a caller enables it.
#pragma once
#include "common.h"
#include <vector>

namespace hgp {

enum KernelId : int {
    KID_RATE_G8 = 0,   // k_rate_group<8, 64>: rating, groups of 8 lanes
    KID_RATE_G16,      // k_rate_group<16, 256>
    KID_RATE_G64,      // k_rate_group<64, 1024>
    KID_RATE_BLOCK,    // k_rate_block (LDS and global tables)
    KID_GAINS,         // k_gains: LP best moves, all degree classes
    KID_LP_FAST,       // k_lp_fast: whole-pair approvals
    KID_LP_PAIRS,      // k_lp_pairs: sorted pair walk, a workgroup per over-budget block pair
    KID_LP_UPDATE,     // k_lp_update_movers: Lambda / Lambda1 / objective of touched nets
    KID_HUB_INSERT,    // k_hub_insert: hub ratings into global tables
    KID_HUB_ARGMAX,    // k_hub_argmax: best target of each table slice
    KID_HUB_LDS,       // k_hub_lds: hub ratings in one workgroup's LDS table
    KID_COUNT
};

struct Timing {
    uint32_t mask = 0;         // kernels whose launches are timed
    bool account = false;      // run the byte-accounting kernels
    uint64_t *acc_dev = nullptr;   // device [KID_COUNT] byte accumulators
    uint32_t *marks = nullptr;     // device stamp arrays for accounting
    size_t marks_len = 0;          // entries per stamp array
    uint32_t stamp = 0;
    std::vector<hipEvent_t> pool;  // free events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[KID_COUNT];
    uint64_t launches[KID_COUNT] = {};
    double acc_host[KID_COUNT] = {};  // bytes counted on the host (sizes known there)
    uint64_t acc_launches[KID_COUNT] = {};
    uint32_t every = 1, phase = 0;     // time launch j of a kernel only when j % every == phase
    uint64_t seen[KID_COUNT] = {};     // launches of each kernel since the last sampling change
};

Timing &timing();

// Records an event pair around the enclosed launch when kernel `kid` is timed.
struct TimedLaunch {
    int kid;
    hipStream_t st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TimedLaunch(int k, hipStream_t s);
    ~TimedLaunch();
};

inline bool accounting(int kid) { return timing().account && (timing().mask >> kid & 1u); }

}  // namespace hgp
