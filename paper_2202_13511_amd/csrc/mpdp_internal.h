// Internal interface between the host runtime (mpdp_host.cpp) and the gfx950
// kernels (mpdp_kernels.hip).  Not part of the public C-ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "mpdp.h"

namespace mpdp {

constexpr int kMaxRel = 32;

// Query information as the kernels read it.  Built on the host, uploaded
// once per call (about 17 KB), staged into LDS by every workgroup.
struct DevGraph {
    uint32_t n, m, is_tree, cost_model;
    uint32_t adj[kMaxRel];            // bit u of adj[v]: edge (u, v)
    uint32_t tree_parent_bit[kMaxRel];// tree joins rooted at relation 0: bit of parent, 0 at the root
    uint32_t tree_desc[kMaxRel];      // tree joins: relations of the subtree rooted at v
    uint32_t nbr_byte[4][256];        // neighbours of a set, one table per byte of the bitmap
    double card[kMaxRel];
    double base_cost[kMaxRel];        // cost of scanning relation v under the chosen model
    double sel[kMaxRel * kMaxRel];    // sel[u * 32 + v], symmetric, 0 without an edge
    uint32_t binom[33 * 33];          // C(a, b) at [a * 33 + b]
};

// Dense memo, indexed by the relation-set bitmap.
struct MemoPtrs {
    double *cost;
    double *card;
    uint32_t *left;
    uint8_t *op;
};

// Device-side counters, cleared by the init kernel.
struct Counters {
    uint32_t level_count[34];   // connected sets found at each level
    uint32_t extract_error;     // nonzero if plan extraction met an inconsistent memo
    uint32_t pad;
    unsigned long long evaluated; // Alg. 3 candidates (general path)
    unsigned long long ccp;       // unordered csg-cmp pairs (general path)
};

hipError_t launch_init(const DevGraph *g, uint32_t n, MemoPtrs memo, Counters *cnt, hipStream_t s);
hipError_t launch_filter(const DevGraph *g, uint32_t k, uint64_t ncand, uint32_t *list, Counters *cnt,
                         hipStream_t s);
hipError_t launch_eval_tree(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand,
                            const uint32_t *list, const Counters *cnt, MemoPtrs memo, hipStream_t s);
hipError_t launch_eval_general(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand,
                               const uint32_t *list, Counters *cnt, MemoPtrs memo, hipStream_t s);
hipError_t launch_extract(const DevGraph *g, uint32_t n, MemoPtrs memo, mpdp_plan_node *plan,
                          double *root_cost, Counters *cnt, hipStream_t s);

}  // namespace mpdp
