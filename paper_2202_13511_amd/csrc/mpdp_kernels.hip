// gfx950 kernels of the MPDP level loop (Section 5, Alg. 5):
//   k_init          memo init + base-relation fill
//   k_level_tree    one level of Alg. 2 (tree join graphs): unrank, filter
//                   and evaluate fused, one lane per connected set
//   k_filter        unrank the k-subsets and keep the connected ones
//   k_eval_general  Alg. 3 (block-based enumeration): one wave64 per set
//   k_extract       rebuild the plan tree from the memo
//
// Everything is integer bitmap work plus a few IEEE binary64 operations per
// join pair; nothing here is a dense contraction, so no MFMA.  Compiled with
// -ffp-contract=off so every cost expression rounds exactly as written.
//
// Memo layout: level-compact.  The entry of S sits at
// level_off[|S|] + colex(S), so one DP level is one contiguous slab and sets
// evaluated together (consecutive colex ranks) gather from neighbouring
// entries of the level below.
#include <hip/hip_runtime.h>

#include "mpdp_device.h"
#include "mpdp_internal.h"

namespace mpdp {
namespace {

// ---------------------------------------------------------------- kernels

__global__ void k_init(const DevGraph *g, uint32_t n, MemoPtrs M, Counters *cnt) {
    const uint32_t t = threadIdx.x;
    if (t < n) {  // colex({t}) = t, level 1 starts at 1
        const uint64_t at = g->lds.loff[1] + t;
        M.cost[at] = g->lds.bcost[t];
        M.card[at] = g->lds.card[t];
        M.left[at] = 0;
        M.op[at] = MPDP_OP_SCAN;
    }
    uint32_t *words = reinterpret_cast<uint32_t *>(cnt);
    for (uint32_t i = t; i < sizeof(Counters) / 4; i += blockDim.x) words[i] = 0;
}

// The ranges of nw wave-sized pieces of a level that this wave walks (w0,
// w0 + ws, ... below we).  Workgroups are dealt to the eight XCDs round
// robin (workgroup b runs on XCD b mod 8).  When the grid divides evenly,
// each XCD sweeps its own contiguous eighth of the level's ranks, so the
// neighbouring colex ranks of level k-1 that those sets gather sit in one
// XCD's L2.
__device__ __forceinline__ void wave_ranges(uint64_t nw, uint64_t &w0, uint64_t &ws, uint64_t &we) {
    if (gridDim.x & 7u) {
        w0 = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
        ws = (uint64_t)gridDim.x * kWaves;
        we = nw;
    } else {
        const uint64_t x = blockIdx.x & 7u;
        w0 = nw * x / 8 + (uint64_t)(blockIdx.x >> 3) * kWaves + (threadIdx.x >> 6);
        ws = (uint64_t)(gridDim.x >> 3) * kWaves;
        we = nw * (x + 1) / 8;
    }
}

// One DP level of a tree join graph, Alg. 5's unrank, filter, evaluate,
// prune and scatter fused.  Each wave walks ranges of 64 * kTreeChunk colex
// ranks (kTreeChunk consecutive ranks per lane: unrank the first, then the
// same-popcount successor), appends the connected sets to its LDS ring in
// rank order, and evaluates 64 of them at a time, one per lane, so no lane
// idles on a disconnected candidate.
template <int CM, int kTreeChunk, bool kCompact, bool kFlat>
__global__ __launch_bounds__(kBlock) void k_level_tree(const DevGraph *g, uint32_t k, uint64_t ncand,
                                                       Counters *cnt, MemoPtrs M) {
    // the LDS image up to the first 32 selectivities: a tree join reads no
    // more (n - 1 <= 31 edges, and no neighbour tables)
    __shared__ __align__(16) unsigned char lds_tree[kTreeLdsBytes];
    __shared__ uint32_t ring_all[kWaves][kTreeRing];
    __shared__ uint32_t ring_bsum_all[kWaves][kTreeRing];
    stage_graph_prefix(g, lds_tree, kTreeLdsBytes);
    const LdsGraph &L = *reinterpret_cast<const LdsGraph *>(lds_tree);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t per_wave = 64ull * kTreeChunk;
    uint64_t w0, ws, we;
    wave_ranges((ncand + per_wave - 1) / per_wave, w0, ws, we);
    const uint32_t found = level_tree_wave<CM, kTreeChunk, kCompact, kTreeRing, tree_sets_per_lane<CM>(),
                                           MPDP_TREE_PAIR_BATCH, false, kFlat, true>(
        L, M, (int)g->n, k, ncand, w0, ws, we, ring_all[threadIdx.x >> 6], ring_bsum_all[threadIdx.x >> 6], lane);
    if (lane == 0 && found) atomicAdd(&cnt->level_count[k], found);
}

// One level of a depth-one tree (a star around relation 0): the connected
// sets {0} + T are enumerated directly by the colex rank of T among the
// (k - 1)-subsets of relations 1 .. n - 1 (no filter), shared evenly by the
// waves (see level_flat_wave).  With the grid a multiple of 8, the
// workgroups of one XCD (blockIdx mod 8) share one eighth of the level, so
// each XCD's L2 sees one contiguous part of the slabs.
template <int CM, int kTreeChunk>
__global__ __launch_bounds__(kBlock) void k_level_flat(const DevGraph *g, uint32_t k, uint64_t nsets, Counters *cnt,
                                                       MemoPtrs M) {
    __shared__ __align__(16) unsigned char lds_tree[kTreeLdsBytes];
    __shared__ uint32_t blk_set[kWaves][flat_block_words(kTreeChunk)];
    __shared__ uint32_t blk_bsum[kWaves][flat_block_words(kTreeChunk)];
    stage_graph_prefix(g, lds_tree, kTreeLdsBytes);
    const LdsGraph &L = *reinterpret_cast<const LdsGraph *>(lds_tree);
    const uint32_t lane = threadIdx.x & 63u;
    uint64_t lo = 0, len = nsets, wave = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6),
             waves = (uint64_t)gridDim.x * kWaves;
    if ((gridDim.x & 7u) == 0) {
        const uint64_t x = blockIdx.x & 7u;
        lo = nsets * x / 8;
        len = nsets * (x + 1) / 8 - lo;
        wave = (uint64_t)(blockIdx.x >> 3) * kWaves + (threadIdx.x >> 6);
        waves = (uint64_t)(gridDim.x >> 3) * kWaves;
    }
    constexpr int R = flat_sets_per_lane<CM>() < kTreeChunk ? flat_sets_per_lane<CM>() : kTreeChunk;
    level_flat_wave<CM, kTreeChunk, R>(L, M, (int)g->n, k, lo, len, wave, waves, blk_set[threadIdx.x >> 6],
                                       blk_bsum[threadIdx.x >> 6], lane);
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAdd(&cnt->level_count[k], (uint32_t)nsets);
}

// Unfused-prune ablation of a tree level (measurement only): the same walk
// and pair costs, but every pair's key is written out (Section 5 before the
// fusion of prune into evaluate) for k_prune.
template <int CM, int kTreeChunk, bool kFlat>
__global__ __launch_bounds__(kBlock) void k_level_tree_unfused(const DevGraph *g, uint32_t k, uint64_t ncand,
                                                               Counters *cnt, MemoPtrs M, PairKey *keys,
                                                               PruneRec *recs) {
    __shared__ __align__(16) unsigned char lds_tree[kTreeLdsBytes];
    __shared__ uint32_t ring_all[kWaves][kTreeRing];
    __shared__ uint32_t ring_bsum_all[kWaves][kTreeRing];
    stage_graph_prefix(g, lds_tree, kTreeLdsBytes);
    const LdsGraph &L = *reinterpret_cast<const LdsGraph *>(lds_tree);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t per_wave = 64ull * kTreeChunk;
    uint64_t w0, ws, we;
    wave_ranges((ncand + per_wave - 1) / per_wave, w0, ws, we);
    const uint32_t found = level_tree_wave<CM, kTreeChunk, true, kTreeRing, 1, MPDP_TREE_PAIR_BATCH, true, kFlat>(
        L, M, (int)g->n, k, ncand, w0, ws, we, ring_all[threadIdx.x >> 6], ring_bsum_all[threadIdx.x >> 6], lane,
        UnfusedOut{keys, recs, &cnt->prune_slots[k]});
    if (lane == 0 && found) atomicAdd(&cnt->level_count[k], found);
}

// Prune of the unfused ablation: one thread per set slot of level k.
__global__ __launch_bounds__(kBlock) void k_prune(const DevGraph *g, uint32_t k, const Counters *cnt, MemoPtrs M,
                                                  const PairKey *keys, const PruneRec *recs) {
    prune_sets<0>(M, k, g->lds.loff[k], cnt->prune_slots[k], keys, recs,
                  (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
}

// A small level of a tree join graph (few candidates, many members per set):
// the same fused steps with kTreeSplitLanes lanes per candidate, so that
// the pairs of a set are gathered at once instead of one lane's batches in
// a row.
template <int CM>
__global__ __launch_bounds__(kBlock) void k_level_tree_split(const DevGraph *g, uint32_t k, uint64_t ncand,
                                                             Counters *cnt, MemoPtrs M) {
    __shared__ __align__(16) unsigned char lds_tree[kTreeLdsBytes];
    stage_graph_prefix(g, lds_tree, kTreeLdsBytes);
    const LdsGraph &L = *reinterpret_cast<const LdsGraph *>(lds_tree);
    const uint32_t lane = threadIdx.x & 63u;
    constexpr uint64_t per_wave = 64 / kTreeSplitLanes;
    uint64_t w0, ws, we;
    wave_ranges((ncand + per_wave - 1) / per_wave, w0, ws, we);
    const uint32_t found =
        level_tree_split_wave<CM, kTreeSplitLanes>(L, M, (int)g->n, k, ncand, w0, ws, we, lane);
    if (lane == 0 && found) atomicAdd(&cnt->level_count[k], found);
}

// Unrank + filter of a block-based level: kFilterChunk consecutive colex
// ranks per lane; sets that induce a tree go to the front of the list, the
// other connected sets to its back.
__global__ __launch_bounds__(kBlock) void k_filter(const DevGraph *g, uint32_t k, uint64_t ncand,
                                                   uint32_t *list, Counters *cnt) {
    __shared__ __align__(16) LdsGraph L;
    stage_graph(g, L);
    const uint32_t n = g->n;
    filter_wave(L, (int)n, k, ncand, (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6),
                (uint64_t)gridDim.x * kWaves, list, L.binom[n * 33 + n / 2], &cnt->level_count[k],
                &cnt->general_count[k], threadIdx.x & 63u, (g->ablate & kAblateDpsub) == 0);
}

// Light work of a block-based level: groups of 64 tree-inducing sets, one
// per lane, then one wave64 per other set.  A set with more than
// kHeavyChunks 16-candidate chunks is handed to k_eval_heavy instead.
template <int CM>
__global__ __launch_bounds__(kBlock) void k_eval_general(const DevGraph *g, uint32_t k, const uint32_t *list,
                                                         uint32_t *heavy, Counters *cnt, MemoPtrs M) {
    __shared__ __align__(16) LdsGraph L;
    __shared__ WaveScratch WS[kWaves];
    __shared__ uint2 SV[kWaves][3 * kSurvCap];
    stage_graph(g, L);
    const uint32_t lane = threadIdx.x & 63u, n = g->n;
    unsigned long long my_ccp = 0, my_eval = 0;
    light_sets<CM>(L, M, list, L.binom[n * 33 + n / 2], cnt->level_count[k], cnt->general_count[k],
                   blockIdx.x * kWaves + (threadIdx.x >> 6), gridDim.x * kWaves, WS[threadIdx.x >> 6], heavy,
                   &cnt->heavy_count[k], lane, my_ccp, my_eval, (g->ablate & kAblateDpsub) != 0, kHeavyChunks,
                   SV[threadIdx.x >> 6]);

    // one atomic per wave for the counters
    for (int off = 32; off >= 1; off >>= 1) {
        my_ccp += (unsigned long long)__shfl_xor((long long)my_ccp, off);
        my_eval += (unsigned long long)__shfl_xor((long long)my_eval, off);
    }
    if (lane == 0 && (my_ccp || my_eval)) {
        atomicAdd(&cnt->ccp, my_ccp);
        atomicAdd(&cnt->evaluated, my_eval);
    }
}

// Alg. 3, heavy sets: one 512-thread workgroup per set, or, when a level
// has fewer heavy sets than workgroups (the top levels of a large cyclic
// query: one set of all relations, then n, ...), `parts` workgroups per
// set, each taking every parts-th run of 512 candidate chunks; their keys
// then go to HeavyPart records for k_heavy_reduce.  Wave 0 of each
// workgroup finds the blocks, all 8 waves share the candidate chunks, and
// the plan keys are reduced through LDS.
template <int CM>
__global__ __launch_bounds__(kHeavyBlock) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_eval_heavy(const DevGraph *g, uint32_t k, const uint32_t *heavy,
                                                            Counters *cnt, MemoPtrs M, HeavyPart *partrec) {
    constexpr int kHW = kHeavyBlock / 64;
    __shared__ __align__(16) LdsGraph L;
    __shared__ WaveScratch W;
    __shared__ SetBlocks sbs;
    __shared__ Key keys[kHW];
    __shared__ uint2 SV[kHW][3 * kSurvCap];
    const uint32_t count = cnt->heavy_count[k];
    const uint32_t parts = heavy_parts(count, gridDim.x);
    if (blockIdx.x >= count * parts) return;  // the whole workgroup, before any barrier
    stage_graph(g, L);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long my_ccp = 0, my_eval = 0;
    for (uint32_t t = blockIdx.x; t < count * parts; t += gridDim.x) {
        const uint32_t h = t / parts, part = t - h * parts;
        const uint32_t S = heavy[h];
        if (wave == 0) {
            const SetBlocks sb = (g->ablate & kAblateDpsub) ? whole_set(S, W, lane, kHeavyBlock)
                                                            : analyze_set(L, S, W, lane, kHeavyBlock);
            if (lane == 0) { sbs = sb; if (part == 0) my_eval += sb.evaluated; }
        }
        __syncthreads();
        const SetBlocks sb = sbs;
        const double cardS = card_of_wave(L, S, threadIdx.x & 63u);
        Key best = worst_key();
        eval_chunks<CM>(L, M, W, S, sb, part * kHeavyBlock + threadIdx.x, parts * kHeavyBlock, cardS, best, my_ccp,
                        SV[wave]);
        best = wave_min(best);
        if (lane == 0) keys[wave] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            Key b = keys[0];
            for (int i = 1; i < kHW; ++i)
                if (key_less(keys[i], b)) b = keys[i];
            if (parts == 1) store_best(M, memo_index(L, S), b, cardS);
            else partrec[t] = HeavyPart{b.c, b.l, b.op, cardS};
        }
        __syncthreads();
    }
    for (int off = 32; off >= 1; off >>= 1) {
        my_ccp += (unsigned long long)__shfl_xor((long long)my_ccp, off);
        my_eval += (unsigned long long)__shfl_xor((long long)my_eval, off);
    }
    if (lane == 0 && (my_ccp || my_eval)) {
        atomicAdd(&cnt->ccp, my_ccp);
        atomicAdd(&cnt->evaluated, my_eval);
    }
}

// The keys of a set split over several heavy workgroups: one thread per
// set combines its parts and writes the memo entry (nothing to do when
// every heavy set had a workgroup of its own).
__global__ __launch_bounds__(64) void k_heavy_reduce(const DevGraph *g, uint32_t k, const uint32_t *heavy,
                                                     const Counters *cnt, MemoPtrs M, const HeavyPart *partrec,
                                                     uint32_t grid) {
    const uint32_t count = cnt->heavy_count[k];
    const uint32_t parts = heavy_parts(count, grid);
    if (parts == 1) return;
    for (uint32_t h = threadIdx.x; h < count; h += blockDim.x) {
        Key b = worst_key();
        for (uint32_t p = 0; p < parts; ++p) {
            const HeavyPart r = partrec[h * parts + p];
            const Key o{r.c, r.l, r.op};
            if (key_less(o, b)) b = o;
        }
        store_best(M, memo_index(g->lds, heavy[h]), b, partrec[h * parts].card);
    }
}

// Rebuild the plan (Section 5: fetched recursively through left/right) in
// post-order with one wave (see extract_plan).
__global__ __launch_bounds__(64) void k_extract(const DevGraph *g, uint32_t n, MemoPtrs M, mpdp_plan_node *plan,
                                                double *root_cost, Counters *cnt) {
    __shared__ uint32_t binom[33 * 33];
    __shared__ uint64_t loff[34];
    __shared__ PlanScratch P;
    for (uint32_t i = threadIdx.x; i < 33 * 33; i += blockDim.x) binom[i] = g->lds.binom[i];
    if (threadIdx.x < 34) loff[threadIdx.x] = g->lds.loff[threadIdx.x];
    __syncthreads();
    if (!extract_plan(binom, loff, M, n, plan, root_cost, P, threadIdx.x, blockDim.x) && threadIdx.x == 0)
        cnt->extract_error = 1;
}

uint32_t grid_for(uint64_t items, uint64_t per_block) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (uint32_t)(b < kMaxGrid ? b : kMaxGrid);
}

}  // namespace

hipError_t launch_init(const DevGraph *g, uint32_t n, MemoPtrs memo, Counters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, g, n, memo, cnt);
    return hipGetLastError();
}

hipError_t launch_filter(const DevGraph *g, uint32_t k, uint64_t ncand, uint32_t *list, Counters *cnt,
                         hipStream_t s) {
    const uint32_t grid = grid_for(ncand, (uint64_t)kBlock * kFilterChunk);
    hipLaunchKernelGGL(k_filter, dim3(grid), dim3(kBlock), 0, s, g, k, ncand, list, cnt);
    return hipGetLastError();
}

hipError_t launch_level_tree(const DevGraph *g, int cost_model, uint32_t n, uint32_t k, uint64_t ncand, bool compact,
                             bool flat, Counters *cnt, MemoPtrs memo, hipStream_t s) {
    // Fewer consecutive ranks per lane on small levels, so that even they
    // spread over some thousands of waves; a persistent-sized grid on large
    // ones, so each workgroup stages the query information once.
    constexpr uint64_t kWantWaves = 1024;
    if (compact && k >= kTreeSplitMinK && ncand <= kTreeSplitMaxCand) {
        const uint64_t per_block = (uint64_t)kWaves * (64 / kTreeSplitLanes);
        uint64_t blocks = (ncand + per_block - 1) / per_block;
        const uint32_t grid = (uint32_t)(blocks > kPersistGrid ? kPersistGrid : blocks);
        if (cost_model == MPDP_COST_COUT)
            hipLaunchKernelGGL(k_level_tree_split<MPDP_COST_COUT>, dim3(grid), dim3(kBlock), 0, s, g, k, ncand, cnt,
                               memo);
        else
            hipLaunchKernelGGL(k_level_tree_split<MPDP_COST_PGLIKE>, dim3(grid), dim3(kBlock), 0, s, g, k, ncand, cnt,
                               memo);
        return hipGetLastError();
    }
    if (compact && flat) {
        // a depth-one tree: its C(n - 1, k - 1) connected sets directly
        const uint64_t nsets = ncand * k / n;
        const int chunk = (cost_model == MPDP_COST_COUT && nsets >= 64ull * 8 * kWantWaves)
                              ? 8
                              : (nsets >= 64ull * 4 * kWantWaves ? 4 : (nsets >= 64ull * 2 * kWantWaves ? 2 : 1));
        const uint64_t blocks = (nsets + (uint64_t)kBlock * chunk - 1) / ((uint64_t)kBlock * chunk);
        const uint32_t cap = cost_model == MPDP_COST_COUT ? kFlatGridCout : kFlatGrid;
        const uint32_t grid = (uint32_t)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
#define MPDP_LEVEL_FLAT(CMV, CH) \
    hipLaunchKernelGGL((k_level_flat<CMV, CH>), dim3(grid), dim3(kBlock), 0, s, g, k, nsets, cnt, memo)
        if (cost_model == MPDP_COST_COUT) {
            if (chunk == 8) MPDP_LEVEL_FLAT(MPDP_COST_COUT, 8);
            else if (chunk == 4) MPDP_LEVEL_FLAT(MPDP_COST_COUT, 4);
            else if (chunk == 2) MPDP_LEVEL_FLAT(MPDP_COST_COUT, 2);
            else MPDP_LEVEL_FLAT(MPDP_COST_COUT, 1);
        } else {
            if (chunk == 4) MPDP_LEVEL_FLAT(MPDP_COST_PGLIKE, 4);
            else if (chunk == 2) MPDP_LEVEL_FLAT(MPDP_COST_PGLIKE, 2);
            else MPDP_LEVEL_FLAT(MPDP_COST_PGLIKE, 1);
        }
#undef MPDP_LEVEL_FLAT
        return hipGetLastError();
    }
    // eight ranks per lane only under C_out: PG-like keeps more registers
    // per set live and measured slower with them
    const int chunk = (cost_model == MPDP_COST_COUT && ncand >= 64ull * 8 * kWantWaves)
                          ? 8
                          : (ncand >= 64ull * 4 * kWantWaves ? 4 : (ncand >= 64ull * 2 * kWantWaves ? 2 : 1));
    uint64_t blocks = (ncand + (uint64_t)kBlock * chunk - 1) / ((uint64_t)kBlock * chunk);
    const uint32_t cap = cost_model == MPDP_COST_COUT ? kPersistGridCout : kPersistGrid;
    const uint32_t grid = (uint32_t)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
    // (a compacted depth-one level went to k_level_flat above; without
    // compaction, the ablation, it keeps the depth-one evaluation)
#define MPDP_LEVEL_TREE(CMV, CH)                                                                        \
    do {                                                                                                \
        if (compact)                                                                                    \
            hipLaunchKernelGGL((k_level_tree<CMV, CH, true, false>), dim3(grid), dim3(kBlock), 0, s, g, k, ncand, cnt, memo); \
        else if (flat)                                                                                  \
            hipLaunchKernelGGL((k_level_tree<CMV, CH, false, true>), dim3(grid), dim3(kBlock), 0, s, g, k, ncand, cnt, memo); \
        else                                                                                            \
            hipLaunchKernelGGL((k_level_tree<CMV, CH, false, false>), dim3(grid), dim3(kBlock), 0, s, g, k, ncand, cnt, memo); \
    } while (0)
    if (cost_model == MPDP_COST_COUT) {
        if (chunk == 8) MPDP_LEVEL_TREE(MPDP_COST_COUT, 8);
        else if (chunk == 4) MPDP_LEVEL_TREE(MPDP_COST_COUT, 4);
        else if (chunk == 2) MPDP_LEVEL_TREE(MPDP_COST_COUT, 2);
        else MPDP_LEVEL_TREE(MPDP_COST_COUT, 1);
    } else {
        if (chunk == 4) MPDP_LEVEL_TREE(MPDP_COST_PGLIKE, 4);
        else if (chunk == 2) MPDP_LEVEL_TREE(MPDP_COST_PGLIKE, 2);
        else MPDP_LEVEL_TREE(MPDP_COST_PGLIKE, 1);
    }
#undef MPDP_LEVEL_TREE
    return hipGetLastError();
}

hipError_t launch_level_tree_unfused(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand, bool flat,
                                     Counters *cnt, MemoPtrs memo, PairKey *keys, PruneRec *recs, hipStream_t s) {
    // the launch shape of the fused kernel on the same level (chunk and grid)
    constexpr uint64_t kWantWaves = 1024;
    const int chunk = ncand >= 64ull * 4 * kWantWaves ? 4 : (ncand >= 64ull * 2 * kWantWaves ? 2 : 1);
    const uint64_t blocks = (ncand + (uint64_t)kBlock * chunk - 1) / ((uint64_t)kBlock * chunk);
    const uint32_t cap = cost_model == MPDP_COST_COUT ? kPersistGridCout : kPersistGrid;
    const uint32_t grid = (uint32_t)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
#define MPDP_UNFUSED(CMV, CH)                                                                                    \
    do {                                                                                                         \
        if (flat)                                                                                                \
            hipLaunchKernelGGL((k_level_tree_unfused<CMV, CH, true>), dim3(grid), dim3(kBlock), 0, s, g, k, ncand, \
                               cnt, memo, keys, recs);                                                           \
        else                                                                                                     \
            hipLaunchKernelGGL((k_level_tree_unfused<CMV, CH, false>), dim3(grid), dim3(kBlock), 0, s, g, k,      \
                               ncand, cnt, memo, keys, recs);                                                    \
    } while (0)
    if (cost_model == MPDP_COST_COUT) {
        if (chunk == 4) MPDP_UNFUSED(MPDP_COST_COUT, 4);
        else if (chunk == 2) MPDP_UNFUSED(MPDP_COST_COUT, 2);
        else MPDP_UNFUSED(MPDP_COST_COUT, 1);
    } else {
        if (chunk == 4) MPDP_UNFUSED(MPDP_COST_PGLIKE, 4);
        else if (chunk == 2) MPDP_UNFUSED(MPDP_COST_PGLIKE, 2);
        else MPDP_UNFUSED(MPDP_COST_PGLIKE, 1);
    }
#undef MPDP_UNFUSED
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prune, dim3(grid_for(ncand, kBlock)), dim3(kBlock), 0, s, g, k, cnt, memo, keys, recs);
    return hipGetLastError();
}

hipError_t launch_eval_general(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand,
                               const uint32_t *list, uint32_t *heavy, Counters *cnt, MemoPtrs memo, HeavyPart *parts,
                               hipStream_t s) {
    // waves stride over the level's sets: a grid of four workgroups per CU
    // stages the LDS image 1024 times instead of once per few sets (clique
    // 18: 7.2 -> 3.7 ms); more workgroups only add launches and staging
    const uint32_t grid = std::min<uint32_t>(grid_for(ncand, kWaves), kGeneralGrid);
    if (cost_model == MPDP_COST_COUT)
        hipLaunchKernelGGL(k_eval_general<MPDP_COST_COUT>, dim3(grid), dim3(kBlock), 0, s, g, k, list, heavy, cnt,
                           memo);
    else
        hipLaunchKernelGGL(k_eval_general<MPDP_COST_PGLIKE>, dim3(grid), dim3(kBlock), 0, s, g, k, list, heavy, cnt,
                           memo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // heavy sets: one per workgroup at a time, two workgroups per CU; a
    // level with fewer heavy sets than workgroups splits each over several
    const uint32_t hgrid = kHeavyGrid;
    if (cost_model == MPDP_COST_COUT)
        hipLaunchKernelGGL(k_eval_heavy<MPDP_COST_COUT>, dim3(hgrid), dim3(kHeavyBlock), 0, s, g, k, heavy, cnt, memo,
                           parts);
    else
        hipLaunchKernelGGL(k_eval_heavy<MPDP_COST_PGLIKE>, dim3(hgrid), dim3(kHeavyBlock), 0, s, g, k, heavy, cnt,
                           memo, parts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_heavy_reduce, dim3(1), dim3(64), 0, s, g, k, heavy, cnt, memo, parts, hgrid);
    return hipGetLastError();
}

hipError_t launch_extract(const DevGraph *g, uint32_t n, MemoPtrs memo, mpdp_plan_node *plan,
                          double *root_cost, Counters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_extract, dim3(1), dim3(64), 0, s, g, n, memo, plan, root_cost, cnt);
    return hipGetLastError();
}

}  // namespace mpdp
