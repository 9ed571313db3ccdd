// Internal interface between the host runtime (mpdp_host.cpp) and the gfx950
// kernels (mpdp_kernels.hip).  Not part of the public C-ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "mpdp.h"

namespace mpdp {

constexpr int kMaxRel = 32;

// Per-workgroup copy of the query information, laid out on the host exactly
// as the kernels keep it in LDS so that staging is a plain 16-byte copy.
// The tree kernel reads only a prefix (kTreeLdsBytes: everything before the
// selectivity rows, plus the rows of a tree's n - 1 <= 31 edges), so the
// selectivity rows and the neighbour tables, which only the block-based
// kernels read in full, come last.
struct LdsImage {
    uint64_t loff[34];                        // memo offset of level k: sum of C(n, j), j < k
    double card[kMaxRel];
    double bcost[kMaxRel];                    // cost of scanning relation v under the model
    double csel[kMaxRel][2];                  // per v: card[v], then sel(lowest u < v adjacent to v, v) (1.0 without one)
    uint32_t ch[4][256];                      // tree joins rooted at 0: children of a set, per byte
    uint32_t lo[kMaxRel][2];                  // per v: bit of its lowest neighbour u < v (0 without one), its other neighbours u < v
    uint32_t adj[kMaxRel];                    // bit u of adj[v]: edge (u, v)
    uint32_t pd[kMaxRel][2];                  // tree joins rooted at 0, per v: bit of its parent (0 at the root),
                                              // then the relations of the subtree rooted at v
    uint32_t selrow[kMaxRel];                 // first sel entry of relation v
    uint32_t binom[33 * 33];                  // C(a, b) at [a * 33 + b]
    uint32_t pad[3];
    double sel[kMaxRel * (kMaxRel - 1) / 2];  // per v: sel(u, v) of edges u < v, u ascending
    uint32_t nb[4][256];                      // neighbours of a set, one table per bitmap byte
};
static_assert(offsetof(LdsImage, csel) % 16 == 0, "(card, sel) pairs are read as 16-byte units");
static_assert(offsetof(LdsImage, lo) % 8 == 0, "lowest-neighbour pairs are read as 8-byte units");
static_assert(offsetof(LdsImage, pd) % 8 == 0, "(parent, subtree) pairs are read as 8-byte units");
static_assert(offsetof(LdsImage, sel) % 16 == 0, "the tree prefix ends on a 16-byte boundary");
constexpr size_t kTreeLdsBytes = offsetof(LdsImage, sel) + 8 * 32;  // the prefix plus 32 selectivities
static_assert(sizeof(LdsImage) % 16 == 0, "LdsImage is copied in 16-byte units");

// Query information as the kernels read it.  Built on the host, uploaded
// once per call.
struct DevGraph {
    LdsImage lds;
    uint32_t n, m, is_tree, cost_model;
    uint32_t ablate;                     // kAblateDpsub: every connected set is one block (DPSUB's enumeration)
    uint32_t flat;                       // tree joins whose tree, rooted at relation 0, has depth one
    uint32_t pad[2];
};

// Memo, level-compact: the entry of a relation set S sits at
// level_off[|S|] + colex(S), colex(S) = sum over the i-th smallest member s_i
// of S (i from 0) of C(s_i, i + 1).  One contiguous slab per level.
struct MemoPtrs {
    double *cost;
    double *card;
    uint32_t *left;
    uint8_t *op;
};

// Device-side counters, cleared by the init kernel.
struct Counters {
    uint32_t level_count[34];   // connected sets found at each level (block-based path: those inducing a tree)
    uint32_t general_count[34]; // block-based path: the other connected sets of each level
    uint32_t heavy_count[34];   // sets handed to the heavy kernel at each level
    uint32_t prune_slots[34];   // unfused-prune ablation: sets whose pair keys were written at each level
    uint32_t extract_error;     // nonzero if plan extraction met an inconsistent memo
    uint32_t pad;
    unsigned long long evaluated; // Alg. 3 candidates (general path)
    unsigned long long ccp;       // unordered csg-cmp pairs (general path)
};

// Batched path (mpdp_batch.hip): one queue entry per workgroup at a time.
// A query is one entry, or, if it is large and cyclic, kTeamSize entries in
// a row: a team of workgroups that share its levels.
struct BatchQueryDev {
    uint32_t n, m, is_tree, cost_model;
    uint64_t card_off, edge_off, plan_off;
    uint32_t sched, out;       // the query's schedule (packed as below); index of its BatchOut
    uint32_t team, member;     // workgroups sharing the query (1: alone); this entry's place among them
    uint32_t team_rec, pad;    // the team's TeamRec (team > 1)
};

// Shared state of one team, zero at the start of a launch.  The first
// member publishes its memo slot, which the whole team uses; the level's
// list counts live here instead of in LDS.
struct TeamRec {
    uint32_t arrive;                 // barrier arrivals so far
    uint32_t slot;                   // workgroup whose slot holds the memo and lists
    uint32_t error;                  // a barrier wait ran out of time
    uint32_t pad;
    uint32_t ntree[24], ngen[24], nheavy[24];  // per level k
    unsigned long long ccp, evaluated;
};

constexpr uint32_t kTeamSize = 8;     // largest team
constexpr uint32_t kTeamMinRel = 17;  // only cyclic queries of at least this many relations may get a team

// Schedule of one query in the batched kernel: bits 0-1 hold log2 of the
// consecutive ranks per lane of a tree query's levels (1, 2 or 4), bits
// 8-23 the number of 16-candidate chunks above which a set of a cyclic
// query is evaluated by the whole workgroup instead of one wave.
constexpr uint32_t kSchedChunkMask = 3u;
constexpr uint32_t kSchedHeavyShift = 8;
constexpr uint32_t kSchedDefault = 2u | (256u << kSchedHeavyShift);

struct BatchOut {
    double cost;
    unsigned long long t_start, t_end;  // device wall clock at the query's start and end
    unsigned long long connected, ccp, evaluated;
    uint32_t error, pad;
};

struct BatchCounters {
    uint32_t next;           // next queue entry to take
    uint32_t entries;        // queue entries of this launch
    unsigned long long t0;   // earliest workgroup start (device wall clock)
};

constexpr uint32_t kBatchMaxRel = 20;      // largest query the batched path takes
static_assert(kBatchMaxRel < 24, "TeamRec holds the counts of levels up to 23");
constexpr uint32_t kBatchWorkgroups = 512; // persistent workgroups (two per CU)

hipError_t launch_batch(int cost_model, uint32_t workgroups, const BatchQueryDev *qs,
                        const uint32_t *edges, const double *cards, const double *sels, const double *bcosts,
                        const uint32_t *binom, char *slots, uint64_t slot_bytes, uint32_t maxn,
                        mpdp_plan_node *plans, BatchOut *out, TeamRec *teams,
                        BatchCounters *bc, hipStream_t s);

hipError_t launch_init(const DevGraph *g, uint32_t n, MemoPtrs memo, Counters *cnt, hipStream_t s);
hipError_t launch_filter(const DevGraph *g, uint32_t k, uint64_t ncand, uint32_t *list, Counters *cnt,
                         hipStream_t s);
constexpr uint32_t kAblateDpsub = 1u;

hipError_t launch_level_tree(const DevGraph *g, int cost_model, uint32_t n, uint32_t k, uint64_t ncand, bool compact,
                             bool flat, Counters *cnt, MemoPtrs memo, hipStream_t s);

// Unfused-prune ablation of a tree level (measurement only): the evaluate
// kernel writes the key of every pair of every connected set (16 bytes,
// k per set, slot-major) and the set's record, a separate prune kernel
// reduces each set's keys and writes its memo entry.  pair_keys holds at
// least C(n, k) * k keys, set_recs C(n, k) records.
struct PruneRec {
    uint32_t rank, set;
    double card;
};
struct PairKey {
    unsigned long long c;
    uint32_t l, op;
};
hipError_t launch_level_tree_unfused(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand, bool flat,
                                     Counters *cnt, MemoPtrs memo, PairKey *pair_keys, PruneRec *set_recs,
                                     hipStream_t s);
// Key and card of one part of a heavy set split over several workgroups.
struct HeavyPart {
    unsigned long long c;
    uint32_t l, op;
    double card;
    double pad;
};
constexpr uint32_t kHeavyGrid = 768;  // workgroups of the heavy-set kernel (three per CU)

// Workgroups per heavy set: one while a level has at least one heavy set
// per workgroup, else as many as share the grid evenly.
__host__ __device__ inline uint32_t heavy_parts(uint32_t count, uint32_t grid) {
    return (count == 0 || count >= grid) ? 1u : grid / count;
}

hipError_t launch_eval_general(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand,
                               const uint32_t *list, uint32_t *heavy, Counters *cnt, MemoPtrs memo, HeavyPart *parts,
                               hipStream_t s);
hipError_t launch_extract(const DevGraph *g, uint32_t n, MemoPtrs memo, mpdp_plan_node *plan,
                          double *root_cost, Counters *cnt, hipStream_t s);

}  // namespace mpdp
