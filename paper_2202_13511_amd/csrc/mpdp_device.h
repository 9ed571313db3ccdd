// Device-side building blocks of the MPDP kernels (shared by the per-level
// kernels in mpdp_kernels.hip and the batched kernel in mpdp_batch.hip).
// Bitmap set algebra, grow, colex ranks, card(S), the plan key, the Alg. 2
// pair evaluation of one set and the Alg. 3 block analysis and candidate
// loop.  Internal; every function is inlined into its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mpdp_internal.h"

namespace mpdp {
namespace {

constexpr int kBlock = 256;         // threads per workgroup (4 waves of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kFilterChunk = 16;    // consecutive ranks per lane in k_filter (<= 31)
// consecutive ranks per lane in k_level_tree: 1, 2 or 4, and 8 on the
// largest levels under C_out (one unrank per eight candidates)
constexpr int kTreeChunkMax = 8;
constexpr int kRing = 384;          // per-wave ring of the batched kernel (chunks up to 4, one set per lane)
constexpr uint32_t kPersistGrid = 1024;  // workgroups that keep the whole chip busy (4 per CU)
// Tree levels under C_out gather one word per pair: three workgroups per CU
// leave fewer gathers in flight and lose fewer of them from the caches
// (PG-like's two words per pair want the fourth).
#ifndef MPDP_TREE_GRID_COUT
#define MPDP_TREE_GRID_COUT 768
#endif
constexpr uint32_t kPersistGridCout = MPDP_TREE_GRID_COUT;
// Tree levels with at least kTreeSplitMinK members per set (two or more
// batches of gathers for one lane) and at most kTreeSplitMaxCand candidates
// are too small to hide a lane's serial gathers: kTreeSplitLanes lanes take
// each candidate there.
constexpr int kTreeSplitLanes = 8;
constexpr uint32_t kTreeSplitMinK = 8;
constexpr uint64_t kTreeSplitMaxCand = 4096;
#ifndef MPDP_HEAVY_CHUNKS
#define MPDP_HEAVY_CHUNKS 512
#endif
constexpr uint32_t kHeavyChunks = MPDP_HEAVY_CHUNKS;   // above this many 16-candidate chunks a set is heavy
constexpr int kHeavyBlock = 512;         // threads per heavy set
constexpr uint32_t kMaxGrid = 8192; // workgroups per launch (grid-stride beyond)
constexpr uint32_t kGeneralGrid = 1024;  // workgroups of a block-based level's light sets

// Sets a lane evaluates at once in k_level_tree (independent chains,
// interleaved): two under C_out, one under PG-like, whose gathers and
// costs of two sets at once need more registers than pay off.
#ifndef MPDP_TREE_SETS_PER_LANE_COUT
#define MPDP_TREE_SETS_PER_LANE_COUT 2
#endif
constexpr int kTreeSetsMax = MPDP_TREE_SETS_PER_LANE_COUT;
template <int CM>
constexpr int tree_sets_per_lane() { return CM == MPDP_COST_COUT ? MPDP_TREE_SETS_PER_LANE_COUT : 1; }
// per-wave ring of k_level_tree: room for the sets a drain leaves (fewer
// than 64 per lane) and one pass of appends (at most 64 * chunk)
constexpr int kTreeRing = 640;
static_assert(kTreeRing >= 64 * kTreeSetsMax - 1 + 64 * kTreeChunkMax, "ring too small");
// members per batch of the tree pair loop (gathers in flight per lane; the
// batched kernel, which keeps much more state live, takes three) and of the
// card(S) pass (LDS reads in flight)
// depth-one tree levels (k_level_flat): sets per lane and grid caps.  On
// a 25-relation star (ms per query) the C_out cap of 256 / 384 / 512 / 768 /
// 1024 workgroups gave 0.84 / 0.78 / 0.78 / 0.83 / 0.87, and the PG-like
// cap of 512 / 768 / 1024 gave 1.14 / 1.12 / 1.20; four C_out sets per lane,
// or two PG-like ones, gained nothing
#ifndef MPDP_FLAT_SETS_PER_LANE_COUT
#define MPDP_FLAT_SETS_PER_LANE_COUT 2
#endif
#ifndef MPDP_FLAT_SETS_PER_LANE_PG
#define MPDP_FLAT_SETS_PER_LANE_PG 1
#endif
template <int CM>
constexpr int flat_sets_per_lane() {
    return CM == MPDP_COST_COUT ? MPDP_FLAT_SETS_PER_LANE_COUT : MPDP_FLAT_SETS_PER_LANE_PG;
}
#ifndef MPDP_FLAT_GRID_COUT
#define MPDP_FLAT_GRID_COUT 512
#endif
#ifndef MPDP_FLAT_GRID
#define MPDP_FLAT_GRID 768
#endif
constexpr uint32_t kFlatGridCout = MPDP_FLAT_GRID_COUT;
constexpr uint32_t kFlatGrid = MPDP_FLAT_GRID;
#ifndef MPDP_TREE_PAIR_BATCH
#define MPDP_TREE_PAIR_BATCH 4
#endif
#ifndef MPDP_TREE_CARD_BATCH
#define MPDP_TREE_CARD_BATCH 4
#endif

// ---------------------------------------------------------------- bitmaps

__device__ __forceinline__ uint32_t lowbit(uint32_t x) { return x & (0u - x); }
__device__ __forceinline__ int ctz32(uint32_t x) { return __builtin_ctz(x); }
__device__ __forceinline__ int popc32(uint32_t x) { return __builtin_popcount(x); }

// Neighbours of every relation in V (a union of adjacency lists), from four
// byte-indexed tables in LDS: four lookups whatever |V| is.
__device__ __forceinline__ uint32_t nbrs(const uint32_t (*nb)[256], uint32_t V) {
    return nb[0][V & 255u] | nb[1][(V >> 8) & 255u] | nb[2][(V >> 16) & 255u] | nb[3][V >> 24];
}

// grow(source, restriction), Section 3.2.1: every relation of `restriction`
// reachable from `source` inside it.  Frontier expansion, one step per BFS
// level.
__device__ __forceinline__ uint32_t grow(const uint32_t (*nb)[256], uint32_t source,
                                         uint32_t restriction) {
    uint32_t seen = source, frontier = source;
    while (frontier) {
        uint32_t fresh = nbrs(nb, frontier) & restriction & ~seen;
        seen |= fresh;
        frontier = fresh;
    }
    return seen;
}

// Children of every relation in V, for a tree join rooted at relation 0.
__device__ __forceinline__ uint32_t children(const uint32_t (*ch)[256], uint32_t V) {
    return ch[0][V & 255u] | ch[1][(V >> 8) & 255u] | ch[2][(V >> 16) & 255u] | ch[3][V >> 24];
}

// Next bitmap with the same popcount (next k-subset in colex order).
__device__ __forceinline__ uint32_t next_subset(uint32_t x) {
    const uint32_t r = x + lowbit(x);
    return (((r ^ x) >> 2) >> ctz32(x)) | r;  // the divisor lowbit(x) is a power of two
}

// Spread the low bits of j over the set bits of mask (parallel bit deposit).
__device__ __forceinline__ uint32_t deposit(uint32_t j, uint32_t mask) {
    uint32_t r = 0;
    for (uint32_t m = mask; j && m; m &= m - 1, j >>= 1)
        if (j & 1u) r |= lowbit(m);
    return r;
}

// ---------------------------------------------------------------- LDS copy

using LdsGraph = LdsImage;

// Copy the host-built LDS image into the workgroup's LDS.
__device__ __forceinline__ void stage_graph(const DevGraph *g, LdsGraph &L) {
    const uint4 *src = reinterpret_cast<const uint4 *>(&g->lds);
    uint4 *dst = reinterpret_cast<uint4 *>(&L);
    for (uint32_t i = threadIdx.x; i < sizeof(LdsGraph) / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Copy the first `bytes` (a multiple of 16) of the host-built LDS image: the
// tree kernel keeps only that prefix (kTreeLdsBytes) in LDS.
__device__ __forceinline__ void stage_graph_prefix(const DevGraph *g, unsigned char *dst_raw, size_t bytes) {
    const uint4 *src = reinterpret_cast<const uint4 *>(&g->lds);
    uint4 *dst = reinterpret_cast<uint4 *>(dst_raw);
    for (uint32_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}
static_assert(kTreeLdsBytes % 16 == 0, "the tree prefix is copied in 16-byte units");

// Memo index of T: level offset plus colex rank.
__device__ __forceinline__ uint64_t memo_index(const LdsGraph &L, uint32_t T) {
    uint32_t r = 0;
    int i = 1;
    for (uint32_t U = T; U; U &= U - 1, ++i) r += L.binom[ctz32(U) * 33 + i];
    return L.loff[i - 1] + r;
}

// Colex unrank of rank r among the k-subsets of n relations: relations from
// n - 1 down, relation c is the next member (i still to place) exactly when
// C(c, i) <= r, the largest such c being the first met.  One uniform,
// branch-free step per relation; C(c, i) = 0 for c < i takes the last
// members once r has reached 0.
__device__ __forceinline__ uint32_t colex_unrank(const uint32_t *binom, int n, int k, uint32_t r) {
    uint32_t S = 0;
    int i = k;
#pragma unroll 4
    for (int c = n - 1; c >= 0; --c) {
        const uint32_t t = binom[c * 33 + i];
        const bool take = (i > 0) & (t <= r);
        r -= take ? t : 0u;
        S |= take ? (1u << c) : 0u;
        i -= take ? 1 : 0;
    }
    return S;
}

// colex_unrank that also returns bsum = sum over the members s_i of S of
// C(s_i, i) (i from 0), read with C(c, i) as its neighbour in the table.
// For the same-popcount successor S' of S, bsum(S') = bsum(S) + t - 1
// where t is the length of the lowest run of ones of S: the run's members
// p .. p+t-1 at places 0 .. t-1 contribute sum_{i<t} C(p+i, i) = C(p+t, t-1)
// (hockey stick), which is exactly what member p+t at place t-1 contributes
// to S', whose places 0 .. t-2 hold members 0 .. t-2 at C(i, i) = 1 each.
__device__ __forceinline__ uint32_t colex_unrank_b(const uint32_t *binom, int n, int k, uint32_t r, uint32_t &bsum) {
    uint32_t S = 0, b = 0;
    int i = k;
#pragma unroll 4
    for (int c = n - 1; c >= 0; --c) {
        const uint32_t at = (uint32_t)(c * 33 + (i > 0 ? i - 1 : 0));
        const uint32_t t0 = binom[at], t1 = binom[at + 1];  // C(c, i - 1), C(c, i)
        const bool take = (i > 0) & (t1 <= r);
        r -= take ? t1 : 0u;
        b += take ? t0 : 0u;
        S |= take ? (1u << c) : 0u;
        i -= take ? 1 : 0;
    }
    bsum = b;
    return S;
}

// bsum of the same-popcount successor of S (see colex_unrank_b).
__device__ __forceinline__ uint32_t next_bsum(uint32_t S, uint32_t bsum) {
    const uint32_t run = ~(S >> ctz32(S));
    return bsum + (uint32_t)ctz32(run | 0x80000000u) - 1u;
}

// ---------------------------------------------------------------- cost

// card(S): product over S ascending of card[v] and of the selectivities of
// the edges from v down to smaller members of S; clamped below at 1.
__device__ __forceinline__ double card_of(const LdsGraph &L, uint32_t S) {
    double c = 1.0;
    for (uint32_t T = S; T; T &= T - 1) {
        const int v = ctz32(T);
        c = c * L.card[v];
        const uint32_t lower = L.adj[v] & ((1u << v) - 1u);
        for (uint32_t U = lower & S; U; U &= U - 1)
            c = c * L.sel[L.selrow[v] + (uint32_t)popc32(lower & (lowbit(U) - 1u))];
    }
    return c < 1.0 ? 1.0 : c;
}

// Plan key: cost bits (non-negative doubles order like their bit patterns),
// then the left relation set, then the operator.
struct Key {
    unsigned long long c;
    uint32_t l;
    uint32_t op;
};

__device__ __forceinline__ bool key_less(const Key &a, const Key &b) {
    if (a.c != b.c) return a.c < b.c;
    if (a.l != b.l) return a.l < b.l;
    return a.op < b.op;
}

__device__ __forceinline__ Key worst_key() { return Key{~0ull, ~0u, ~0u}; }

__device__ __forceinline__ void offer(Key &best, double cost, uint32_t left, uint32_t op) {
    Key k{(unsigned long long)__double_as_longlong(cost), left, op};
    if (key_less(k, best)) best = k;
}

// Cost both orientations of the csg-cmp pair (A, B) of S, whose memo entries
// sit at ia and ib, and keep the best.
template <int CM>
__device__ __forceinline__ void eval_pair(const MemoPtrs &M, uint32_t A, uint32_t B, uint64_t ia, uint64_t ib,
                                          double cardS, Key &best) {
    const double cA = M.cost[ia], cB = M.cost[ib];
    const double base = cA + cB;
    if (CM == MPDP_COST_COUT) {
        // symmetric: both orientations cost the same, the smaller left wins
        offer(best, base + cardS, A < B ? A : B, MPDP_OP_JOIN);
    } else {
        const double kA = M.card[ia], kB = M.card[ib];
        const double out = 0.01 * cardS;
        const double hjA = ((base + 0.0125 * kB) + 0.0025 * kA) + out;  // A outer, B hashed
        const double nlA = (base + (0.0025 * kA) * kB) + out;
        const double hjB = ((base + 0.0125 * kA) + 0.0025 * kB) + out;  // B outer, A hashed
        const double nlB = (base + (0.0025 * kB) * kA) + out;
        if (hjA <= nlA) offer(best, hjA, A, MPDP_OP_HASH); else offer(best, nlA, A, MPDP_OP_NESTLOOP);
        if (hjB <= nlB) offer(best, hjB, B, MPDP_OP_HASH); else offer(best, nlB, B, MPDP_OP_NESTLOOP);
    }
}

__device__ __forceinline__ void store_best(const MemoPtrs &M, uint64_t at, const Key &b, double cardS) {
    M.cost[at] = __longlong_as_double((long long)b.c);
    M.card[at] = cardS;
    M.left[at] = b.l;
    M.op[at] = (uint8_t)b.op;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cost both orientations of the pair (A, B) of S from the two sides' memo
// values and keep the best.
template <int CM>
__device__ __forceinline__ void eval_vals(uint32_t A, uint32_t B, double cA, double cB, double kA, double kB,
                                          double cardS, Key &best) {
    const double base = cA + cB;
    if (CM == MPDP_COST_COUT) {
        offer(best, base + cardS, A < B ? A : B, MPDP_OP_JOIN);
    } else {
        const double out = 0.01 * cardS;
        const double hjA = ((base + 0.0125 * kB) + 0.0025 * kA) + out;  // A outer, B hashed
        const double nlA = (base + (0.0025 * kA) * kB) + out;
        const double hjB = ((base + 0.0125 * kA) + 0.0025 * kB) + out;  // B outer, A hashed
        const double nlB = (base + (0.0025 * kB) * kA) + out;
        if (hjA <= nlA) offer(best, hjA, A, MPDP_OP_HASH); else offer(best, nlA, A, MPDP_OP_NESTLOOP);
        if (hjB <= nlB) offer(best, hjB, B, MPDP_OP_HASH); else offer(best, nlB, B, MPDP_OP_NESTLOOP);
    }
}


// Key order with the operator compared only where it can decide (not under
// C_out, whose offers all carry one operator).
template <int CM>
__device__ __forceinline__ bool key_less_sel(unsigned long long ac, uint32_t al, uint32_t aop, const Key &b) {
    if (CM == MPDP_COST_COUT) return (ac < b.c) | ((ac == b.c) & (al < b.l));
    return (ac < b.c) | ((ac == b.c) & ((al < b.l) | ((al == b.l) & (aop < b.op))));
}

template <int CM>
__device__ __forceinline__ void offer_if(bool on, Key &best, double cost, uint32_t left, uint32_t op) {
    const unsigned long long c = (unsigned long long)__double_as_longlong(cost);
    const bool take = on & key_less_sel<CM>(c, left, op, best);
    best.c = take ? c : best.c;
    best.l = take ? left : best.l;
    if (CM != MPDP_COST_COUT) best.op = take ? op : best.op;
}

// One pass over the k members of R tree-inducing sets S[r] of one level
// (R independent chains per lane, interleaved): bsum = sum of C(s_i, i),
// and card(S) in card_of's order (members ascending, each card then the
// selectivities of its edges to smaller members, ascending).  The edge to
// v's lowest smaller neighbour comes from the (card, sel) pair of v (times
// an exact 1.0 when that neighbour is outside S); v's other smaller
// neighbours in S, which a tree seldom has, go through the sel row.
// Members go in batches whose LDS reads are all issued before the products
// use them (slots past k read relation 31's entries, C(31, i) and a
// (1.0, 1.0) pair, and are masked); the products stay in member order.
template <int R>
__device__ __forceinline__ void tree_bsum_card_n(const LdsGraph &L, const uint32_t *S, uint32_t k, uint32_t *bsum,
                                                 double *cardS) {
    constexpr int kB = MPDP_TREE_CARD_BATCH;
    double c[R];
    uint32_t b[R], T[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { c[r] = 1.0; b[r] = 0; T[r] = S[r]; }
    for (uint32_t i0 = 0; i0 < k; i0 += kB) {
        int vv[R][kB];
        uint32_t bb[R][kB];
        double2 cs[R][kB];
        uint2 lo[R][kB];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                vv[r][u] = ctz32(T[r] | 0x80000000u);
                T[r] &= T[r] - 1;
                bb[r][u] = L.binom[vv[r][u] * 33 + i0 + u];
                cs[r][u] = *reinterpret_cast<const double2 *>(L.csel[vv[r][u]]);
                lo[r][u] = *reinterpret_cast<const uint2 *>(L.lo[vv[r][u]]);
            }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (i0 + (uint32_t)u < k) {  // uniform: every set of the level has k members
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    b[r] += bb[r][u];
                    c[r] = c[r] * cs[r][u].x;
                    c[r] = c[r] * ((S[r] & lo[r][u].x) ? cs[r][u].y : 1.0);
                    const uint32_t rest = lo[r][u].y & S[r];
                    if (rest) {
                        const int v = vv[r][u];
                        const uint32_t lower = L.adj[v] & ((1u << v) - 1u);
                        for (uint32_t U = rest; U; U &= U - 1)
                            c[r] = c[r] * L.sel[L.selrow[v] + (uint32_t)popc32(lower & (lowbit(U) - 1u))];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bsum[r] = b[r];
        cardS[r] = c[r] < 1.0 ? 1.0 : c[r];
    }
}

__device__ __forceinline__ void tree_bsum_card(const LdsGraph &L, uint32_t S, uint32_t k, uint32_t &bsum,
                                               double &cardS) {
    tree_bsum_card_n<1>(L, &S, k, &bsum, &cardS);
}

// card(S) of R tree-inducing sets of one level, as tree_bsum_card_n without
// the colex sums.
template <int R>
__device__ __forceinline__ void tree_card_n(const LdsGraph &L, const uint32_t *S, uint32_t k, double *cardS) {
    constexpr int kB = MPDP_TREE_CARD_BATCH;
    double c[R];
    uint32_t T[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { c[r] = 1.0; T[r] = S[r]; }
    for (uint32_t i0 = 0; i0 < k; i0 += kB) {
        int vv[R][kB];
        double2 cs[R][kB];
        uint2 lo[R][kB];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                vv[r][u] = ctz32(T[r] | 0x80000000u);
                T[r] &= T[r] - 1;
                cs[r][u] = *reinterpret_cast<const double2 *>(L.csel[vv[r][u]]);
                lo[r][u] = *reinterpret_cast<const uint2 *>(L.lo[vv[r][u]]);
            }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (i0 + (uint32_t)u < k) {  // uniform: every set of the level has k members
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    c[r] = c[r] * cs[r][u].x;
                    c[r] = c[r] * ((S[r] & lo[r][u].x) ? cs[r][u].y : 1.0);
                    const uint32_t rest = lo[r][u].y & S[r];
                    if (rest) {
                        const int v = vv[r][u];
                        const uint32_t lower = L.adj[v] & ((1u << v) - 1u);
                        for (uint32_t U = rest; U; U &= U - 1)
                            c[r] = c[r] * L.sel[L.selrow[v] + (uint32_t)popc32(lower & (lowbit(U) - 1u))];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) cardS[r] = c[r] < 1.0 ? 1.0 : c[r];
}

// Alg. 2 for R connected sets of one level per lane (R independent
// chains, interleaved; see eval_tree_set for one).  Every set has k members
// and k is the same on all lanes, so the member loops run a uniform k times
// (scalar branches only).  Members go in batches of kPairBatch whose memo
// gathers are all issued before any is used; the topmost member stays in
// its batch as an empty slot (A = 0) that gathers a harmless singleton and
// offers nothing.
// Where eval_tree_sets leaves its results: fused (the default), each set's
// best key goes to the memo; unfused (the prune ablation), every pair's key
// goes to keys[slot[r] * k + member index] and the set's record to
// recs[slot[r]], for a separate prune kernel.
struct TreeSink {
    PairKey *keys = nullptr;
    PruneRec *recs = nullptr;
    uint32_t slot[2] = {0, 0};
};

template <int CM, int R, int kPairBatch = MPDP_TREE_PAIR_BATCH, bool kUnfused = false, bool kBatchKeys = false>
__device__ __forceinline__ void eval_tree_sets(const LdsGraph &L, const MemoPtrs &M, const uint32_t *S,
                                               const uint32_t *bsum, uint32_t k, uint64_t off_k,
                                               const double *__restrict__ cost_km1,
                                               const double *__restrict__ card_km1,
                                               const TreeSink &sink = TreeSink{}) {
    // each set's bsum = sum of C(s_i, i) comes with it from the filter, and
    // its own colex rank sum C(s_i, i + 1) accumulates in pa below
    double cardS[R];
    tree_card_n<R>(L, S, k, cardS);
    // C_out offers carry one operator, so the running best starts with it
    // and the operator never decides
    Key best[R];
    double bc[R];  // kBatchKeys (C_out): running smallest cost, +inf before the first pair
    uint32_t pa[R], pb[R], T[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        best[r] = worst_key();
        bc[r] = __builtin_inf();
        if (CM == MPDP_COST_COUT) best[r].op = MPDP_OP_JOIN;
        pa[r] = pb[r] = 0;
        T[r] = S[r];
    }
    for (uint32_t i0 = 0; i0 < k; i0 += kPairBatch) {
        // members i0 .. i0 + kPairBatch - 1 (slots past k read relation
        // 31's entries, which exist, and are masked); all LDS reads of the
        // batch are issued before any is used
        uint32_t Av[R][kPairBatch], rk[R][kPairBatch], ba[R][kPairBatch], bb[R][kPairBatch];
        int mv[R][kPairBatch];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < kPairBatch; ++u) {
                const uint32_t i = i0 + (uint32_t)u;
                const bool live = i < k;
                const int m = ctz32(T[r] | 0x80000000u);
                T[r] &= T[r] - 1;
                mv[r][u] = m;
                bb[r][u] = L.binom[m * 33 + i];
                ba[r][u] = L.binom[m * 33 + i + 1];
                const uint2 pd = *reinterpret_cast<const uint2 *>(L.pd[m]);  // parent bit, subtree
                const uint32_t on = (uint32_t)(live & ((S[r] & pd.x) != 0));
                Av[r][u] = pd.y & S[r] & (0u - on);
            }
        uint32_t multi = 0;  // a side of two or more relations in this batch
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < kPairBatch; ++u) {
                // a slot past the last member gathers entry 0
                const bool live = i0 + (uint32_t)u < k;
                pb[r] += bb[r][u];
                rk[r][u] = live ? pa[r] + (bsum[r] - pb[r]) : 0u;
                pa[r] += live ? ba[r][u] : 0u;
                multi |= Av[r][u] & (Av[r][u] - 1u);
            }
        double cA[R][kPairBatch], cB[R][kPairBatch], kA[R][kPairBatch], kB[R][kPairBatch];
        if (__ballot(multi != 0) == 0) {
            // every pair of the batch, on every lane, splits off one relation
            // (always so on a star): one straight run of gathers, all in
            // flight together
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) {
                    cB[r][u] = cost_km1[rk[r][u]];
                    if (CM != MPDP_COST_COUT) kB[r][u] = card_km1[rk[r][u]];
                }
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) {
                    const int m = mv[r][u] & 31;
                    cA[r][u] = L.bcost[m];
                    kA[r][u] = L.card[m];
                }
        } else {
            // some side has two or more relations: its memo index and its
            // complement's come from colex sums (LDS only); then every slot
            // gathers both sides in one straight run (a singleton side
            // gathers its partner's entry again and takes its own values
            // from LDS)
            uint64_t ia[R][kPairBatch], ib[R][kPairBatch];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) {
                    const uint32_t A = Av[r][u];
                    const bool single = (A & (A - 1)) == 0;
                    ib[r][u] = single ? L.loff[k - 1] + rk[r][u] : memo_index(L, S[r] ^ A);
                    ia[r][u] = single ? ib[r][u] : memo_index(L, A);
                }
            double gA[R][kPairBatch], hA[R][kPairBatch];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) {
                    cB[r][u] = M.cost[ib[r][u]];
                    gA[r][u] = M.cost[ia[r][u]];
                    if (CM != MPDP_COST_COUT) {
                        kB[r][u] = M.card[ib[r][u]];
                        hA[r][u] = M.card[ia[r][u]];
                    }
                }
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) {
                    const uint32_t A = Av[r][u];
                    const bool single = (A & (A - 1)) == 0;
                    const int m = ctz32(A | 0x80000000u) & 31;
                    cA[r][u] = single ? L.bcost[m] : gA[r][u];
                    if (CM != MPDP_COST_COUT) kA[r][u] = single ? L.card[m] : hA[r][u];
                }
        }
        if (CM == MPDP_COST_COUT && kBatchKeys && !kUnfused) {
            // the batch's keys without per-pair branches: the smallest cost
            // of the batch and the running best, then the smallest left set
            // among the pairs that reach it (the key order); a slot without
            // a pair costs +inf, and a connected set has at least one pair
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double c[kPairBatch];
                uint32_t l[kPairBatch];
                double mn = bc[r];
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) {
                    const uint32_t A = Av[r][u], B = S[r] ^ A;
                    c[u] = A != 0 ? (cA[r][u] + cB[r][u]) + cardS[r] : __builtin_inf();
                    l[u] = A < B ? A : B;
                    mn = __builtin_fmin(mn, c[u]);
                }
                uint32_t nl = bc[r] == mn ? best[r].l : ~0u;
#pragma unroll
                for (int u = 0; u < kPairBatch; ++u) nl = min(nl, c[u] == mn ? l[u] : ~0u);
                bc[r] = mn;
                best[r].l = nl;
            }
            continue;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < kPairBatch; ++u) {
                const uint32_t A = Av[r][u], B = S[r] ^ A;
                const bool on = A != 0;
                const double base = cA[r][u] + cB[r][u];
                if (kUnfused) {
                    // this pair's best orientation alone, written out
                    Key one = worst_key();
                    if (CM == MPDP_COST_COUT) {
                        one.op = MPDP_OP_JOIN;
                        offer_if<CM>(on, one, base + cardS[r], A < B ? A : B, MPDP_OP_JOIN);
                    } else {
                        const double out = 0.01 * cardS[r];
                        const double hjA = ((base + 0.0125 * kB[r][u]) + 0.0025 * kA[r][u]) + out;
                        const double nlA = (base + (0.0025 * kA[r][u]) * kB[r][u]) + out;
                        const double hjB = ((base + 0.0125 * kA[r][u]) + 0.0025 * kB[r][u]) + out;
                        const double nlB = (base + (0.0025 * kB[r][u]) * kA[r][u]) + out;
                        const bool hA = hjA <= nlA, hB = hjB <= nlB;
                        offer_if<CM>(on, one, hA ? hjA : nlA, A, hA ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
                        offer_if<CM>(on, one, hB ? hjB : nlB, B, hB ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
                    }
                    if (i0 + (uint32_t)u < k)
                        sink.keys[(uint64_t)sink.slot[r] * k + i0 + (uint32_t)u] = PairKey{one.c, one.l, one.op};
                    continue;
                }
                if (CM == MPDP_COST_COUT) {
                    offer_if<CM>(on, best[r], base + cardS[r], A < B ? A : B, MPDP_OP_JOIN);
                } else {
                    const double out = 0.01 * cardS[r];
                    const double hjA = ((base + 0.0125 * kB[r][u]) + 0.0025 * kA[r][u]) + out;  // A outer, B hashed
                    const double nlA = (base + (0.0025 * kA[r][u]) * kB[r][u]) + out;
                    const double hjB = ((base + 0.0125 * kA[r][u]) + 0.0025 * kB[r][u]) + out;  // B outer, A hashed
                    const double nlB = (base + (0.0025 * kB[r][u]) * kA[r][u]) + out;
                    const bool hA = hjA <= nlA, hB = hjB <= nlB;
                    offer_if<CM>(on, best[r], hA ? hjA : nlA, A, hA ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
                    offer_if<CM>(on, best[r], hB ? hjB : nlB, B, hB ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
                }
            }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (CM == MPDP_COST_COUT && kBatchKeys && !kUnfused) best[r].c = (unsigned long long)__double_as_longlong(bc[r]);
        if (kUnfused) sink.recs[sink.slot[r]] = PruneRec{pa[r], S[r], cardS[r]};
        else store_best(M, off_k + pa[r], best[r], cardS[r]);
    }
}

// Prune step of the unfused ablation: one lane per set slot of level k
// reduces the k pair keys of its set (members without a pair hold the worst
// key) and writes the memo entry.
template <int CM>
__device__ __forceinline__ void prune_sets(const MemoPtrs &M, uint32_t k, uint64_t off_k, uint32_t count,
                                           const PairKey *keys, const PruneRec *recs, uint64_t i0, uint64_t stride) {
    for (uint64_t i = i0; i < count; i += stride) {
        Key best = worst_key();
        for (uint32_t j = 0; j < k; ++j) {
            const PairKey p = keys[i * k + j];
            const Key o{p.c, p.l, p.op};
            if (key_less(o, best)) best = o;
        }
        const PruneRec rec = recs[i];
        store_best(M, off_k + rec.rank, best, rec.card);
    }
}

// Alg. 2 for one connected S of a tree join graph.  With the tree rooted at
// relation 0, removing the edge (parent(c), c) of G[S] gives the pair
// (desc(c) & S, S minus that) for every c in S whose parent is in S, which
// is every member but the topmost one.  When desc(c) & S = {c} the
// complement's colex rank follows from prefix sums,
// rank(S - s_j) = sum_{i<j} C(s_i, i+1) + sum_{i>j} C(s_i, i), and the
// singleton's cost and card come from LDS.
template <int CM, int kPairBatch = MPDP_TREE_PAIR_BATCH>
__device__ __forceinline__ void eval_tree_set(const LdsGraph &L, const MemoPtrs &M, uint32_t S, uint32_t bsum,
                                              uint32_t k, uint64_t off_k, const double *__restrict__ cost_km1,
                                              const double *__restrict__ card_km1) {
    eval_tree_sets<CM, 1, kPairBatch>(L, M, &S, &bsum, k, off_k, cost_km1, card_km1);
}

// Alg. 2 when the join tree, rooted at relation 0, has depth one: every
// other relation is a leaf on relation 0 (a star around relation 0).  Every
// connected set of two or more relations then holds relation 0 as its
// smallest member, and the edge (0, m) of each other member m gives the
// pair ({m}, S - {m}); so no subtree lookups, no topmost member to skip, and
// every pair splits off one relation whose cost and card come from LDS.
// card(S) is tree_card_n's product with its conditions settled: each member
// ascending multiplies its card, then its selectivity to relation 0 (1.0
// for relation 0 itself), and no member has another smaller neighbour.
// A batch's keys are reduced without per-offer branches: the smallest cost
// of the batch and the running best first, then the smallest left set among
// the offers that reach it, which is key_less's order (a connected set has
// at least one pair, so the running best's +inf start never survives; under
// PG-like the operator follows from the left set, see flat_batch).  Pairs go
// in batches of kPairBatch (members 1 .. k - 1); only the last batch of a
// set has slots past its last member, and they take no part (skipped under
// C_out, +inf offers under PG-like).
struct FlatBest {
    double c;     // running smallest cost (+inf before the first pair)
    uint32_t l;   // smallest left set at that cost
    uint32_t op;  // its operator (PG-like)
};

template <int CM, int R, int kPairBatch, bool kFull, bool kUnfused>
__device__ __forceinline__ void flat_batch(const LdsGraph &L, const uint32_t *S, const uint32_t *bsum,
                                           uint32_t p0, uint32_t np, const double *cardS,
                                           const double *__restrict__ cost_km1,
                                           const double *__restrict__ card_km1, uint32_t *pa, uint32_t *pb,
                                           uint32_t *T, FlatBest *best, const TreeSink &sink, uint32_t k) {
    int mv[R][kPairBatch];
    uint32_t rk[R][kPairBatch], ba[R][kPairBatch], bb[R][kPairBatch];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            const uint32_t i = p0 + (uint32_t)u + 1u;  // member index; slots past k read valid rows
            const int m = ctz32(T[r] | 0x80000000u);
            T[r] &= T[r] - 1;
            mv[r][u] = m;
            bb[r][u] = L.binom[m * 33 + i];
            ba[r][u] = L.binom[m * 33 + i + 1];
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            const bool live = kFull || p0 + (uint32_t)u < np;  // uniform
            pb[r] += bb[r][u];
            rk[r][u] = live ? pa[r] + (bsum[r] - pb[r]) : 0u;  // a dead slot gathers entry 0
            pa[r] += live ? ba[r][u] : 0u;
        }
    double cB[R][kPairBatch], kB[R][kPairBatch];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            cB[r][u] = cost_km1[rk[r][u]];
            if (CM != MPDP_COST_COUT) kB[r][u] = card_km1[rk[r][u]];
        }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double c[kPairBatch];
        uint32_t l[kPairBatch];
        double pc[2 * kPairBatch];  // PG-like offers: cost, left set, operator
        uint32_t pl[2 * kPairBatch], po[2 * kPairBatch];
        double mn = best[r].c;
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            const bool live = kFull || p0 + (uint32_t)u < np;
            const int m = mv[r][u] & 31;
            const uint32_t A = 1u << m, B = S[r] ^ A;
            const double cA = L.bcost[m];
            const double base = cA + cB[r][u];
            if (CM == MPDP_COST_COUT) {
                c[u] = base + cardS[r];
                l[u] = A < B ? A : B;
                if (kUnfused) {
                    if (live)
                        sink.keys[(uint64_t)sink.slot[r] * k + p0 + (uint32_t)u + 1u] =
                            PairKey{(unsigned long long)__double_as_longlong(c[u]), l[u], MPDP_OP_JOIN};
                } else if (live) {
                    mn = __builtin_fmin(mn, c[u]);
                }
            } else {
                const double kA = L.card[m];
                const double out = 0.01 * cardS[r];
                const double hjA = ((base + 0.0125 * kB[r][u]) + 0.0025 * kA) + out;  // A outer, B hashed
                const double nlA = (base + (0.0025 * kA) * kB[r][u]) + out;
                const double hjB = ((base + 0.0125 * kA) + 0.0025 * kB[r][u]) + out;  // B outer, A hashed
                const double nlB = (base + (0.0025 * kB[r][u]) * kA) + out;
                const bool hA = hjA <= nlA, hB = hjB <= nlB;
                if (kUnfused) {
                    Key one = worst_key();
                    offer_if<CM>(true, one, hA ? hjA : nlA, A, hA ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
                    offer_if<CM>(true, one, hB ? hjB : nlB, B, hB ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
                    if (live) sink.keys[(uint64_t)sink.slot[r] * k + p0 + (uint32_t)u + 1u] = PairKey{one.c, one.l, one.op};
                } else {
                    // both orientations; a slot past the last member offers +inf
                    pc[2 * u] = live ? (hA ? hjA : nlA) : __builtin_inf();
                    pl[2 * u] = A;
                    po[2 * u] = hA ? MPDP_OP_HASH : MPDP_OP_NESTLOOP;
                    pc[2 * u + 1] = live ? (hB ? hjB : nlB) : __builtin_inf();
                    pl[2 * u + 1] = B;
                    po[2 * u + 1] = hB ? MPDP_OP_HASH : MPDP_OP_NESTLOOP;
                    mn = __builtin_fmin(mn, __builtin_fmin(pc[2 * u], pc[2 * u + 1]));
                }
            }
        }
        if (CM == MPDP_COST_COUT && !kUnfused) {
            uint32_t nl = best[r].c == mn ? best[r].l : ~0u;
#pragma unroll
            for (int u = 0; u < kPairBatch; ++u) {
                const bool live = kFull || p0 + (uint32_t)u < np;
                if (live) nl = min(nl, c[u] == mn ? l[u] : ~0u);
            }
            best[r].c = mn;
            best[r].l = nl;
        }
        if (CM != MPDP_COST_COUT && !kUnfused) {
            // PG-like: the smallest cost, then the smallest left set at it;
            // the left sets of a set's offers all differ (one relation, or
            // all but one, and both only for two relations, which have one
            // pair), so that left set names one offer, whose operator is
            // taken: the key order (cost, left set, operator)
            uint32_t nl = best[r].c == mn ? best[r].l : ~0u;
#pragma unroll
            for (int o = 0; o < 2 * kPairBatch; ++o) nl = min(nl, pc[o] == mn ? pl[o] : ~0u);
            uint32_t nop = (best[r].c == mn && best[r].l == nl) ? best[r].op : ~0u;
#pragma unroll
            for (int o = 0; o < 2 * kPairBatch; ++o) nop = min(nop, (pc[o] == mn && pl[o] == nl) ? po[o] : ~0u);
            best[r].c = mn;
            best[r].l = nl;
            best[r].op = nop;
        }
    }
}

template <int CM, int R, int kPairBatch = MPDP_TREE_PAIR_BATCH, bool kUnfused = false>
__device__ __forceinline__ void eval_flat_sets(const LdsGraph &L, const MemoPtrs &M, const uint32_t *S,
                                               const uint32_t *bsum, uint32_t k, uint64_t off_k,
                                               const double *__restrict__ cost_km1,
                                               const double *__restrict__ card_km1,
                                               const TreeSink &sink = TreeSink{}) {
    constexpr int kCB = MPDP_TREE_CARD_BATCH;
    double cardS[R];
    {
        double c[R];
        uint32_t T[R];
#pragma unroll
        for (int r = 0; r < R; ++r) { c[r] = 1.0; T[r] = S[r]; }
        for (uint32_t i0 = 0; i0 < k; i0 += kCB) {
            double2 cs[R][kCB];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < kCB; ++u) {
                    const int v = ctz32(T[r] | 0x80000000u);
                    T[r] &= T[r] - 1;
                    cs[r][u] = *reinterpret_cast<const double2 *>(L.csel[v]);
                }
#pragma unroll
            for (int u = 0; u < kCB; ++u)
                if (i0 + (uint32_t)u < k)  // uniform
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        c[r] = c[r] * cs[r][u].x;
                        c[r] = c[r] * cs[r][u].y;
                    }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) cardS[r] = c[r] < 1.0 ? 1.0 : c[r];
    }
    // relation 0 is member 0: C(0, 0) = 1 goes to pb, C(0, 1) = 0 to pa
    uint32_t pa[R], pb[R], T[R];
    FlatBest best[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        pa[r] = 0;
        pb[r] = 1;
        T[r] = S[r] & ~1u;
        best[r].c = __builtin_inf();
        best[r].l = ~0u;
        best[r].op = ~0u;
        if (kUnfused) sink.keys[(uint64_t)sink.slot[r] * k] = PairKey{~0ull, ~0u, ~0u};  // member 0 has no pair
    }
    const uint32_t np = k - 1;
    uint32_t p0 = 0;
    for (; p0 + kPairBatch <= np; p0 += kPairBatch)
        flat_batch<CM, R, kPairBatch, true, kUnfused>(L, S, bsum, p0, np, cardS, cost_km1, card_km1, pa, pb, T, best,
                                                      sink, k);
    if (p0 < np)
        flat_batch<CM, R, kPairBatch, false, kUnfused>(L, S, bsum, p0, np, cardS, cost_km1, card_km1, pa, pb, T,
                                                       best, sink, k);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (kUnfused) {
            sink.recs[sink.slot[r]] = PruneRec{pa[r], S[r], cardS[r]};
        } else if (CM == MPDP_COST_COUT) {
            store_best(M, off_k + pa[r], Key{(unsigned long long)__double_as_longlong(best[r].c), best[r].l,
                                             MPDP_OP_JOIN}, cardS[r]);
        } else {
            store_best(M, off_k + pa[r], Key{(unsigned long long)__double_as_longlong(best[r].c), best[r].l,
                                             best[r].op}, cardS[r]);
        }
    }
}

// eval_tree_set with the pairs of S spread over a group of P lanes (P
// divides 64, groups are P consecutive lanes, all active together): lane
// `sub` costs members sub, sub + P, ... (at most 32 / P of them, every
// gather issued before any is used), then the group's keys are combined by
// exchanges within the group and its first lane stores the entry.  Every
// lane walks all k members for the colex ranks, so this pays only where a
// level has too few sets to hide the gathers of a lane-per-set walk.
template <int CM, int P>
__device__ __forceinline__ void eval_tree_set_split(const LdsGraph &L, const MemoPtrs &M, uint32_t S, uint32_t rank,
                                                    uint32_t k, uint32_t sub, uint64_t off_k,
                                                    const double *__restrict__ cost_km1,
                                                    const double *__restrict__ card_km1) {
    constexpr int kSlots = 32 / P;
    uint32_t bsum;
    double cardS;
    tree_bsum_card(L, S, k, bsum, cardS);
    uint32_t Av[kSlots], rk[kSlots];
#pragma unroll
    for (int u = 0; u < kSlots; ++u) Av[u] = rk[u] = 0u;
    uint32_t pa = 0, pb = 0, T = S;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        if ((uint32_t)i < k) {
            const int m = ctz32(T);
            T &= T - 1;
            pb += L.binom[m * 33 + i];
            const uint32_t r = pa + (bsum - pb);  // colex rank of S - {m} at level k - 1
            pa += L.binom[m * 33 + i + 1];
            if ((uint32_t)(i % P) == sub && (S & L.pd[m][0])) {
                Av[i / P] = L.pd[m][1] & S;
                rk[i / P] = r;
            }
        }
    }
    double cA[kSlots], cB[kSlots], kA[kSlots], kB[kSlots];
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        const uint32_t A = Av[u];
        if ((A & (A - 1)) == 0) {  // a singleton, or an empty slot (gathers entry 0)
            cB[u] = cost_km1[rk[u]];
            if (CM != MPDP_COST_COUT) kB[u] = card_km1[rk[u]];
            const int m = ctz32(A | 0x80000000u);
            cA[u] = L.bcost[m & 31];
            kA[u] = L.card[m & 31];
        } else {
            const uint64_t ia = memo_index(L, A), ib = memo_index(L, S ^ A);
            cA[u] = M.cost[ia];
            cB[u] = M.cost[ib];
            if (CM != MPDP_COST_COUT) {
                kA[u] = M.card[ia];
                kB[u] = M.card[ib];
            }
        }
    }
    Key best = worst_key();
    if (CM == MPDP_COST_COUT) best.op = MPDP_OP_JOIN;
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        const uint32_t A = Av[u], B = S ^ A;
        const bool on = A != 0;
        const double base = cA[u] + cB[u];
        if (CM == MPDP_COST_COUT) {
            offer_if<CM>(on, best, base + cardS, A < B ? A : B, MPDP_OP_JOIN);
        } else {
            const double out = 0.01 * cardS;
            const double hjA = ((base + 0.0125 * kB[u]) + 0.0025 * kA[u]) + out;  // A outer, B hashed
            const double nlA = (base + (0.0025 * kA[u]) * kB[u]) + out;
            const double hjB = ((base + 0.0125 * kA[u]) + 0.0025 * kB[u]) + out;  // B outer, A hashed
            const double nlB = (base + (0.0025 * kB[u]) * kA[u]) + out;
            const bool hA = hjA <= nlA, hB = hjB <= nlB;
            offer_if<CM>(on, best, hA ? hjA : nlA, A, hA ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
            offer_if<CM>(on, best, hB ? hjB : nlB, B, hB ? MPDP_OP_HASH : MPDP_OP_NESTLOOP);
        }
    }
    // a lane without pairs keeps the worst key, which never wins over a
    // real offer; the key order is total, so the combining order is free
#pragma unroll
    for (int d = 1; d < P; d <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)best.c, d, P);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(best.c >> 32), d, P);
        Key o;
        o.c = ((unsigned long long)hi << 32) | lo;
        o.l = (uint32_t)__shfl_xor((int)best.l, d, P);
        o.op = (uint32_t)__shfl_xor((int)best.op, d, P);
        if (key_less(o, best)) best = o;
    }
    if (sub == 0) store_best(M, off_k + rank, best, cardS);
}


// Key reduction across the 64 lanes of a wave, returned to every lane:
// four DPP row shifts leave each row's minimum in its last lane, and the
// four row minima are combined from scalar copies.
template <int kCtrl>
__device__ __forceinline__ Key dpp_row_shr(const Key &b) {
    // a lane whose source is outside its row keeps its own key
    const uint32_t lo = (uint32_t)b.c, hi = (uint32_t)(b.c >> 32);
    Key o;
    const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, kCtrl, 0xf, 0xf, false);
    const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, kCtrl, 0xf, 0xf, false);
    o.c = ((unsigned long long)ohi << 32) | olo;
    o.l = (uint32_t)__builtin_amdgcn_update_dpp((int)b.l, (int)b.l, kCtrl, 0xf, 0xf, false);
    o.op = (uint32_t)__builtin_amdgcn_update_dpp((int)b.op, (int)b.op, kCtrl, 0xf, 0xf, false);
    return o;
}

__device__ __forceinline__ Key key_at(const Key &b, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b.c, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b.c >> 32), lane);
    return Key{((unsigned long long)hi << 32) | lo, (uint32_t)__builtin_amdgcn_readlane((int)b.l, lane),
               (uint32_t)__builtin_amdgcn_readlane((int)b.op, lane)};
}

__device__ __forceinline__ Key wave_min(Key b) {
    Key o = dpp_row_shr<0x111>(b);  // row_shr:1
    if (key_less(o, b)) b = o;
    o = dpp_row_shr<0x112>(b);      // row_shr:2
    if (key_less(o, b)) b = o;
    o = dpp_row_shr<0x114>(b);      // row_shr:4
    if (key_less(o, b)) b = o;
    o = dpp_row_shr<0x118>(b);      // row_shr:8
    if (key_less(o, b)) b = o;
    Key r = key_at(b, 15);
    const Key r1 = key_at(b, 31), r2 = key_at(b, 47), r3 = key_at(b, 63);
    if (key_less(r1, r)) r = r1;
    if (key_less(r2, r)) r = r2;
    if (key_less(r3, r)) r = r3;
    return r;
}

// Sum over the lanes 0..31 of a wave of 32-bit values (DPP row scans, then
// the two row totals), returned to every lane.
__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 15) + (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
}

// memo_index of a set S held by the whole wave: lane v adds the term of
// relation v.
__device__ __forceinline__ uint64_t memo_index_wave(const LdsGraph &L, uint32_t S, uint32_t lane) {
    uint32_t term = 0;
    if (lane < 32 && ((S >> lane) & 1u)) term = L.binom[lane * 33 + popc32(S & ((1u << lane) - 1u)) + 1];
    return L.loff[popc32(S)] + wave_sum32(term);
}

__device__ __forceinline__ double rdlane_f64(double x, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// card(S) for a set S held by the whole wave, the same product in the same
// order as card_of: the factors are loaded by all lanes at once (lane v:
// card[v], adjacency and selectivity row of v; lane j and j + 64: the
// selectivities j and j + 64 in edge order) and multiplied from scalar
// copies.
__device__ __forceinline__ double card_of_wave(const LdsGraph &L, uint32_t S, uint32_t lane) {
    const uint32_t v_l = lane & 31u;
    const double cv = L.card[v_l];
    const uint32_t adjv = L.adj[v_l], rowv = L.selrow[v_l];
    const double s0 = L.sel[lane], s1 = L.sel[lane + 64];
    double c = 1.0;
    for (uint32_t T = S; T; T &= T - 1) {
        const int v = ctz32(T);
        c = c * rdlane_f64(cv, v);
        const uint32_t lower = (uint32_t)__builtin_amdgcn_readlane((int)adjv, v) & ((1u << v) - 1u);
        const uint32_t row = (uint32_t)__builtin_amdgcn_readlane((int)rowv, v);
        for (uint32_t U = lower & S; U; U &= U - 1) {
            const uint32_t j = row + (uint32_t)popc32(lower & (lowbit(U) - 1u));
            const double x = j < 64u ? rdlane_f64(s0, (int)j) : j < 128u ? rdlane_f64(s1, (int)(j - 64u)) : L.sel[j];
            c = c * x;
        }
    }
    return c < 1.0 ? 1.0 : c;
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

struct WaveScratch {
    uint32_t blk[32];    // blocks of G[S]
    uint32_t full[32];   // 1 if the block's induced subgraph is complete
    uint32_t cpre[33];   // prefix of candidate chunks per block
};

struct SetBlocks {
    uint32_t A;             // cut vertices of G[S]
    uint32_t total_chunks;  // candidate chunks over all blocks, 2^shift candidates each
    uint32_t shift;
    uint32_t chunks16;      // chunks at 16 candidates each (decides light or heavy in the batched kernel)
    uint32_t work16;        // the same with a sparse block's chunks weighted 1/16: most of its
                            // candidates fall to the per-chunk neighbourhood test (per-level kernels)
    unsigned long long evaluated;  // Alg. 3 candidates of S: sum over blocks of 2^b - 2
};

// Blocks of G[S] for one connected S, computed by one wave:
//  1. a depth-first search from the lowest relation, uniform across the wave:
//     the adjacency of the current relation comes from its lane by readlane,
//     lane v records its parent and, on the way back, its subtree D(v);
//  2. non-tree edges of a depth-first tree join a relation to an ancestor,
//     so the parent p of v separates D(v) from the rest of S exactly when
//     every neighbour of D(v) outside it is p (the lowpoint test); such a v
//     is the top of one block;
//  3. the block of top v is p plus D(v) without the subtrees of the tops
//     below v; the cut vertices are the parents of tops, the root only when
//     it has two or more children.
// The block list, completeness flags and candidate-chunk prefix go to W.
// The half of a block's candidates that hold its lowest relation is cut into
// chunks of 2^shift, with the smallest shift (up to 4) that leaves at most
// `budget` chunks, so that the candidates of a small set still spread over
// all the lanes that take part.
// DPSUB's enumeration (ablation): S itself is the only block, no cut vertex.
__device__ SetBlocks whole_set(uint32_t S, WaveScratch &W, int lane, uint32_t budget) {
    const int k = popc32(S);
    const uint32_t half = (1u << (k - 1)) - 1u;
    uint32_t shift = 4;
    for (uint32_t sh = 0; sh <= 4; ++sh)
        if (((half + (1u << sh) - 1u) >> sh) <= budget) { shift = sh; break; }
    const uint32_t chunks = (half + (1u << shift) - 1u) >> shift;
    if (lane == 0) {
        W.blk[0] = S;
        W.full[0] = 0;
        W.cpre[0] = 0;
        W.cpre[1] = chunks;
    }
    return SetBlocks{0u, chunks, shift, (half + 15u) >> 4, (half + 15u) >> 4, (1ull << k) - 2ull};
}

__device__ SetBlocks analyze_set(const LdsGraph &L, uint32_t S, WaveScratch &W, int lane, uint32_t budget) {
    const bool mine = lane < 32 && ((S >> lane) & 1u);
    const uint32_t adjS = mine ? (L.adj[lane] & S) : 0u;

    // 0. a complete G[S] (every set of a clique) is one complete block with
    // no cut vertex: what the search below finds, without its serial steps
    if (__ballot(mine && (adjS | (1u << lane)) != S) == 0ull) {
        const int k = popc32(S);
        const uint32_t half = (1u << (k - 1)) - 1u;
        const uint32_t c[5] = {half, (half + 1u) >> 1, (half + 3u) >> 2, (half + 7u) >> 3, (half + 15u) >> 4};
        const uint32_t shift = c[0] <= budget ? 0u : c[1] <= budget ? 1u : c[2] <= budget ? 2u : c[3] <= budget ? 3u : 4u;
        if (lane == 0) {
            W.blk[0] = S;
            W.full[0] = 1u;
            W.cpre[0] = 0u;
            W.cpre[1] = c[shift];
        }
        return SetBlocks{0u, c[shift], shift, c[4], c[4], (1ull << k) - 2ull};
    }

    // 1. depth-first search: k - 1 steps down, k - 1 back up, one final test
    const uint32_t root = (uint32_t)ctz32(S);
    uint32_t par = 0, desc = mine ? (1u << lane) : 0u;
    uint32_t cur = root, seen = 1u << root;
    for (int step = 0; step < 2 * kMaxRel; ++step) {
        const uint32_t next = rdlane(adjS, (int)cur) & ~seen;
        if (next) {
            const uint32_t c = (uint32_t)ctz32(next);
            if (lane == (int)c) par = cur;
            seen |= 1u << c;
            cur = c;
        } else {
            if (cur == root) break;
            const uint32_t p = rdlane(par, (int)cur);
            const uint32_t d = rdlane(desc, (int)cur);
            if (lane == (int)p) desc |= d;
            cur = p;
        }
    }

    // 2. lowpoint test, one neighbourhood lookup per lane
    const bool child = mine && lane != (int)root;
    const uint32_t outside = child ? (nbrs(L.nb, desc) & S & ~desc) : 0u;
    const bool top = child && outside == (1u << par);
    const uint32_t T = (uint32_t)__ballot(top);
    const uint32_t rootkids = (uint32_t)__popcll(__ballot(child && par == root));

    // 3. blocks and cut vertices
    uint32_t A = 0, inner = 0;
    for (uint32_t U = T; U; U &= U - 1) {
        const uint32_t t = (uint32_t)ctz32(U);
        A |= 1u << rdlane(par, (int)t);
        const uint32_t dt = rdlane(desc, (int)t);
        if (lane != (int)t && ((desc >> t) & 1u)) inner |= dt;
    }
    if (rootkids < 2) A &= ~(1u << root);
    const uint32_t myblk = top ? ((desc & ~inner) | (1u << par)) : 0u;

    // per-block candidates with the lowest relation (a top lane owns its block)
    uint32_t half = 0, complete = 0;
    if (top) {
        const int bs = popc32(myblk);
        half = (1u << (bs - 1)) - 1u;
        complete = bs <= 3;  // a bridge or a triangle
    }
    {   // larger blocks: complete iff every member is adjacent to all the others
        uint32_t d2 = 0;
        for (uint32_t U = S; U; U &= U - 1) {
            const int v = ctz32(U);
            const uint32_t a = rdlane(adjS, v);
            if ((myblk >> v) & 1u) d2 += (uint32_t)popc32(a & myblk);
        }
        const int bs = popc32(myblk);
        if (top && bs > 3) complete = d2 == (uint32_t)(bs * (bs - 1));
    }
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, w4 = 0;
    for (uint32_t U = T; U; U &= U - 1) {
        const uint32_t h = rdlane(half, ctz32(U));
        c0 += h;
        c1 += (h + 1u) >> 1;
        c2 += (h + 3u) >> 2;
        c3 += (h + 7u) >> 3;
        c4 += (h + 15u) >> 4;
        w4 += rdlane(complete, ctz32(U)) ? (h + 15u) >> 4 : (h + 255u) >> 8;
    }
    const uint32_t shift = c0 <= budget ? 0u : c1 <= budget ? 1u : c2 <= budget ? 2u : c3 <= budget ? 3u : 4u;
    const uint32_t round = (1u << shift) - 1u;
    uint32_t acc = 0, idx = 0;
    unsigned long long evaluated = 0;
    for (uint32_t U = T; U; U &= U - 1, ++idx) {
        const int t = ctz32(U);
        if (lane == t) { W.blk[idx] = myblk; W.full[idx] = complete; W.cpre[idx] = acc; }
        acc += (rdlane(half, t) + round) >> shift;
        evaluated += (1ull << popc32(rdlane(myblk, t))) - 2ull;
    }
    if (lane == 0) W.cpre[idx] = acc;
    return SetBlocks{A, acc, shift, c4, w4, evaluated};
}

// Colex ranks of Sl and of S - Sl in one pass over the members of S.
// A member's place on its side is a popcount, so the table reads of four
// members at a time are issued together (slots past the last member read
// C(0, 1) and are masked).
__device__ __forceinline__ void split_ranks(const LdsGraph &L, uint32_t S, uint32_t Sl, uint32_t &rl, uint32_t &rr) {
    const uint32_t Sr = S & ~Sl;
    uint32_t a = 0, b = 0;
    for (uint32_t T = S; T;) {
        uint32_t c[4], on[4], left[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t v = (uint32_t)ctz32(T | 0x80000000u), below = (1u << v) - 1u;
            on[u] = T != 0u;
            left[u] = (Sl >> v) & 1u;
            const uint32_t place = (uint32_t)popc32((left[u] ? Sl : Sr) & below) + 1u;
            c[u] = L.binom[on[u] ? v * 33u + place : 1u];
            T &= T - 1u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a += (on[u] && left[u]) ? c[u] : 0u;
            b += (on[u] && !left[u]) ? c[u] : 0u;
        }
    }
    rl = a;
    rr = b;
}

// The pair of S from one Alg. 3 candidate whose two sides are connected:
// S_left = grow(lb, S - rb) (lb when the block has no cut vertex of S), and
// S_right = S - S_left, costed in both orientations.
template <int CM>
__device__ __forceinline__ void eval_lb(const LdsGraph &L, const MemoPtrs &M, uint32_t S, uint32_t A, int k,
                                        uint32_t lb, uint32_t rb, double cardS, Key &best,
                                        unsigned long long &ccp) {
    ++ccp;
    const uint32_t Sl = (lb & A) ? grow(L.nb, lb, S & ~rb) : lb;
    uint32_t rl, rr;
    split_ranks(L, S, Sl, rl, rr);
    const int kl = popc32(Sl);
    eval_pair<CM>(M, Sl, S ^ Sl, L.loff[kl] + rl, L.loff[k - kl] + rr, cardS, best);
}

// The CCP check of a candidate (lb, rb) of a block: G[lb] and G[rb]
// connected (they are adjacent because the block is).
__device__ __forceinline__ bool ccp_lb(const LdsGraph &L, uint32_t lb, uint32_t rb) {
    return grow(L.nb, lowbit(lb), lb) == lb && grow(L.nb, lowbit(rb), rb) == rb;
}

// Buffers of one wave, kSurvCap entries each: the candidates that pass the
// neighbourhood tests (checked 64 at a time), the ones that pass the CCP
// check (costed 64 at a time), and the live chunks (tested 64 at a time).
constexpr uint32_t kSurvCap = 128;

// One candidate per lane (`ok`: it passed the CCP check) appended to the
// wave's buffer of valid pairs `vb` (vfill < 64 entries there, uniform);
// 64 of them are costed together once there are.
template <int CM>
__device__ __forceinline__ void push_valid(const LdsGraph &L, const MemoPtrs &M, uint32_t S, uint32_t A, int k,
                                           uint2 e, bool ok, uint2 *vb, uint32_t &vfill, uint32_t lane,
                                           unsigned long long below_me, double cardS, Key &best,
                                           unsigned long long &ccp) {
    const unsigned long long m = __ballot(ok);
    if (ok) vb[vfill + (uint32_t)__popcll(m & below_me)] = e;
    vfill += (uint32_t)__popcll(m);
    wave_sync_lds();
    if (vfill >= 64u) {
        const uint2 v = vb[vfill - 64u + lane];
        vfill -= 64u;
        wave_sync_lds();
        eval_lb<CM>(L, M, S, A, k, v.x, v.y, cardS, best, ccp);
    }
}

// Pass 1 of a live chunk from the chunk buffer (entry: the deposit of its
// shared members, and its block index << 8 | its candidate count): the
// neighbourhoods of the shared parts are looked up once and those of the
// 16 low combinations built from four adjacency rows, so the isolated-member
// test is a few register operations per candidate (candidate t takes the
// members of low4 named by the bits of t, a compile-time choice).  Returns
// the surviving candidates as a 16-bit mask with the chunk's H, RH, low4.
__device__ __forceinline__ void chunk_pass1(const LdsGraph &L, const WaveScratch &W, uint2 e, uint32_t &pend,
                                            uint32_t &H, uint32_t &RH, uint32_t &low4, uint4 &edges) {
    const uint32_t b = W.blk[e.y >> 8], lim = e.y & 255u;
    const uint32_t lo = lowbit(b), rest = b ^ lo;
    const uint32_t m0 = lowbit(rest), r1 = rest ^ m0, m1 = lowbit(r1), r2 = r1 ^ m1, m2 = lowbit(r2),
                   m3 = lowbit(r2 ^ m2);
    low4 = m0 | m1 | m2 | m3;
    const uint32_t a0 = L.adj[ctz32(m0)], a1 = L.adj[ctz32(m1)], a2 = L.adj[ctz32(m2)], a3 = L.adj[ctz32(m3)];
    H = lo | e.x;
    RH = (rest & ~low4) & ~e.x;
    const uint32_t NH = nbrs(L.nb, H), NRH = nbrs(L.nb, RH);
    pend = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const uint32_t ls = ((t & 1) ? m0 : 0u) | ((t & 2) ? m1 : 0u) | ((t & 4) ? m2 : 0u) | ((t & 8) ? m3 : 0u);
        const uint32_t nl = ((t & 1) ? a0 : 0u) | ((t & 2) ? a1 : 0u) | ((t & 4) ? a2 : 0u) | ((t & 8) ? a3 : 0u);
        const uint32_t nr = ((t & 1) ? 0u : a0) | ((t & 2) ? 0u : a1) | ((t & 4) ? 0u : a2) | ((t & 8) ? 0u : a3);
        const uint32_t lb = H | ls, rb = RH | (low4 ^ ls);
        const bool dead = ((lb & (lb - 1)) && (lb & ~(NH | nl))) || ((rb & (rb - 1)) && (rb & ~(NRH | nr)));
        pend |= (!dead && (uint32_t)t < lim) ? (1u << t) : 0u;
    }
    // for the survivors' edge test (place_survivors): twice the edges inside
    // H and inside RH, each low member's edges to H and to RH (one byte
    // each), and which pairs of low members are adjacent (bit i*4+j)
    uint32_t eH2 = 0, eR2 = 0;
    if (pend) {
        for (uint32_t X = H; X;) {
            uint32_t a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = X ? L.adj[ctz32(X)] : 0u;
                X &= X - 1u;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) eH2 += (uint32_t)popc32(a[u] & H);
        }
        for (uint32_t X = RH; X;) {
            uint32_t a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = X ? L.adj[ctz32(X)] : 0u;
                X &= X - 1u;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) eR2 += (uint32_t)popc32(a[u] & RH);
        }
    }
    const uint32_t cH = (uint32_t)popc32(a0 & H) | ((uint32_t)popc32(a1 & H) << 8) |
                        ((uint32_t)popc32(a2 & H) << 16) | ((uint32_t)popc32(a3 & H) << 24);
    const uint32_t cR = (uint32_t)popc32(a0 & RH) | ((uint32_t)popc32(a1 & RH) << 8) |
                        ((uint32_t)popc32(a2 & RH) << 16) | ((uint32_t)popc32(a3 & RH) << 24);
    const uint32_t adjl = ((a0 & m1) ? 0x0002u : 0u) | ((a0 & m2) ? 0x0004u : 0u) | ((a0 & m3) ? 0x0008u : 0u) |
                          ((a1 & m2) ? 0x0040u : 0u) | ((a1 & m3) ? 0x0080u : 0u) | ((a2 & m3) ? 0x0800u : 0u);
    edges = make_uint4(eH2 | (eR2 << 16), cH, cR, adjl);
}

// Every lane's surviving candidates (pend) into the wave's survivor buffer
// (as many as fit), then 64 at a time out of it through the CCP check, until
// every lane has placed its own.
template <int CM>
__device__ __forceinline__ void place_survivors(const LdsGraph &L, const MemoPtrs &M, uint32_t S, uint32_t A, int k,
                                                uint32_t pend, uint32_t H, uint32_t RH, uint32_t low4, uint4 edges,
                                                uint2 *sv, uint32_t &fill, uint32_t &vfill, uint32_t lane,
                                                unsigned long long below_me, double cardS, Key &best,
                                                unsigned long long &ccp) {
    // a connected side of m members has at least m - 1 edges, and a
    // disconnected side without cycles has fewer: most survivors that fail
    // the CCP check fail this count, from per-chunk sums and no lookups
    {
        const uint32_t eH2 = edges.x & 0xffffu, eR2 = edges.x >> 16, nH = (uint32_t)popc32(H),
                       nR = (uint32_t)popc32(RH);
        for (uint32_t Lm = pend; Lm; Lm &= Lm - 1) {
            const uint32_t t = (uint32_t)ctz32(Lm), r = ~t & 15u;
            // low members named by t (left) and the others (right)
            uint32_t el = eH2, er = eR2, il = 0, ir = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                el += ((t >> i) & 1u) ? 2u * ((edges.y >> (8 * i)) & 255u) : 0u;
                er += ((r >> i) & 1u) ? 2u * ((edges.z >> (8 * i)) & 255u) : 0u;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = i + 1; j < 4; ++j) {
                    const uint32_t adj = (edges.w >> (i * 4 + j)) & 1u;
                    il += (adj && ((t >> i) & 1u) && ((t >> j) & 1u)) ? 2u : 0u;
                    ir += (adj && ((r >> i) & 1u) && ((r >> j) & 1u)) ? 2u : 0u;
                }
            const uint32_t nl = nH + (uint32_t)popc32(t), nr = nR + (uint32_t)popc32(r);
            if (el + il + 2u < 2u * nl || er + ir + 2u < 2u * nr) pend &= ~(1u << t);
        }
    }
    while (__ballot(pend != 0) != 0ull) {
        const uint32_t c = (uint32_t)popc32(pend);  // at most 16
        uint32_t before = 0;
#pragma unroll
        for (int bt = 0; bt < 5; ++bt)
            before += (uint32_t)__popcll(__ballot((c >> bt) & 1u) & below_me) << bt;
        const uint32_t total = (uint32_t)__shfl((int)(before + c), 63);
        uint32_t slot = fill + before;
        for (uint32_t Lm = pend; Lm && slot < kSurvCap; Lm &= Lm - 1, ++slot) {
            const uint32_t t = (uint32_t)ctz32(Lm);
            const uint32_t ls = deposit(t, low4);
            sv[slot] = make_uint2(H | ls, RH | (low4 ^ ls));
            pend &= ~(1u << t);
        }
        fill = min(kSurvCap, fill + total);
        wave_sync_lds();
        while (fill >= 64u) {
            const uint2 e = sv[fill - 64u + lane];
            fill -= 64u;
            wave_sync_lds();
            push_valid<CM>(L, M, S, A, k, e, ccp_lb(L, e.x, e.y), sv + kSurvCap, vfill, lane, below_me, cardS, best,
                           ccp);
        }
    }
}

// Alg. 3 candidates of S over the chunks ch = first, first + stride, ... of
// its blocks: for each block-local lb holding the block's lowest relation
// (lb != block, so each unordered pair is met once and both orientations
// are costed) the CCP check, then S_left and S_right (eval_lb).  A thread's
// next chunk in the same block is `stride` chunks on, so its first
// candidate's deposit over the block's members follows by one masked add
// (the holes filled with ones carry through); only a new block needs the
// bit-by-bit deposit.
//
// With chunk tables (the per-level kernels; `first - lane` and `stride`
// multiples of 64, so every wave walks its chunks together, and `sv` the
// wave's survivor buffer): the candidates of a sparse block's chunk that
// pass the neighbourhood tests go to the buffer, and whenever 64 are there
// the wave checks and costs them with every lane busy, instead of each
// lane walking its own few while the others wait.
template <int CM, bool kChunkTables = true>
__device__ __forceinline__ void eval_chunks(const LdsGraph &L, const MemoPtrs &M, const WaveScratch &W, uint32_t S,
                                            const SetBlocks &sb, uint32_t first, uint32_t stride, double cardS,
                                            Key &best, unsigned long long &ccp, uint2 *sv = nullptr) {
    const int k = popc32(S);
    const uint32_t A = sb.A;
    const uint32_t lane = first & 63u;
    const unsigned long long below_me = (1ull << lane) - 1ull;
    int bi = -1;
    uint32_t j0 = 0, hi0 = 0, dstep = 0, fill = 0, vfill = 0, cfill = 0;
    uint2 *cb = sv + 2u * kSurvCap;
    const uint32_t base0 = kChunkTables ? first - lane : first, lane_off = kChunkTables ? lane : 0u;
    for (uint32_t base = base0; base < sb.total_chunks; base += stride) {
        const uint32_t ch = base + lane_off;
        bool alive = false;
        uint2 centry = make_uint2(0u, 0u);
        if (ch < sb.total_chunks) {
            const bool fresh = bi < 0 || ch >= W.cpre[bi + 1];
            if (fresh) {
                bi = bi < 0 ? 0 : bi;
                while (W.cpre[bi + 1] <= ch) ++bi;
            }
            const uint32_t b = W.blk[bi];
            const bool full = W.full[bi] != 0;
            const uint32_t lo = lowbit(b), rest = b ^ lo;
            const uint32_t hb = (1u << (popc32(b) - 1)) - 1u;
            if (fresh) {
                j0 = (ch - W.cpre[bi]) << sb.shift;
                hi0 = deposit(j0, rest);
                // a step that leaves the block's range is never taken: the
                // next chunk is then in a later block
                dstep = deposit(stride << sb.shift, rest);
            } else {
                j0 += stride << sb.shift;
                hi0 = ((hi0 | ~rest) + dstep) & rest;
            }
            const uint32_t j1 = min(j0 + (1u << sb.shift), hb);
            if (kChunkTables && !full && sb.shift == 4 && popc32(rest) >= 5) {
                // 16 candidates share the members of rest above its lowest
                // four (`hi` in lb, the others of that part in rb) and differ
                // in which of those four (low4) they take.  The chunk is dead
                // when a shared member on either side has no neighbour among
                // its side's shared members and low4 (that side then has two
                // or more members in every candidate); a live chunk goes to
                // the wave's chunk buffer (chunk_pass1).
                const uint32_t m0 = lowbit(rest), r1 = rest ^ m0, m1 = lowbit(r1), r2 = r1 ^ m1, m2 = lowbit(r2),
                               m3 = lowbit(r2 ^ m2), low4 = m0 | m1 | m2 | m3;
                const uint32_t N4 = L.adj[ctz32(m0)] | L.adj[ctz32(m1)] | L.adj[ctz32(m2)] | L.adj[ctz32(m3)];
                const uint32_t H = lo | hi0, RH = (rest & ~low4) & ~hi0;  // j0 is a multiple of 16
                const uint32_t NH = nbrs(L.nb, H), NRH = nbrs(L.nb, RH);
                if (!(((H & (H - 1)) && (H & ~(NH | N4))) || ((RH & (RH - 1)) && (RH & ~(NRH | N4))))) {
                    alive = true;
                    centry = make_uint2(hi0, ((uint32_t)bi << 8) | (j1 - j0));
                }
            } else {
                uint32_t sub = hi0;
                for (uint32_t j = j0; j < j1; ++j) {
                    const uint32_t lb = lo | sub, rb = b ^ lb;
                    sub = (sub - rest) & rest;
                    if (!full) {
                        // a connected side of two or more relations has no
                        // member without a neighbour on its side: four table
                        // lookups reject most disconnected candidates of a
                        // sparse block before the breadth-first check
                        if ((lb & (lb - 1)) && (lb & ~nbrs(L.nb, lb))) continue;
                        if ((rb & (rb - 1)) && (rb & ~nbrs(L.nb, rb))) continue;
                        if (grow(L.nb, lo, lb) != lb) continue;
                        if (grow(L.nb, lowbit(rb), rb) != rb) continue;
                    }
                    eval_lb<CM>(L, M, S, A, k, lb, rb, cardS, best, ccp);
                }
            }
        }
        if (!kChunkTables) continue;
        // this round's live chunks into the wave's chunk buffer; once 64
        // are there, each lane tests the 16 candidates of one of them and
        // the survivors go on to the survivor buffer
        const unsigned long long am = __ballot(alive);
        if (alive) cb[cfill + (uint32_t)__popcll(am & below_me)] = centry;
        cfill += (uint32_t)__popcll(am);
        wave_sync_lds();
        if (cfill >= 64u) {
            const uint2 ce = cb[cfill - 64u + lane];
            cfill -= 64u;
            wave_sync_lds();
            uint32_t pend, H, RH, low4;
            uint4 edges;
            chunk_pass1(L, W, ce, pend, H, RH, low4, edges);
            place_survivors<CM>(L, M, S, A, k, pend, H, RH, low4, edges, sv, fill, vfill, lane, below_me, cardS, best,
                                ccp);
        }
    }
    if (kChunkTables) {
        if (cfill != 0u) {
            const uint2 ce = lane < cfill ? cb[lane] : make_uint2(0u, 1u);  // an empty chunk: no candidate
            wave_sync_lds();
            uint32_t pend = 0, H = 0, RH = 0, low4 = 0;
            uint4 edges = make_uint4(0u, 0u, 0u, 0u);
            if (lane < cfill) chunk_pass1(L, W, ce, pend, H, RH, low4, edges);
            place_survivors<CM>(L, M, S, A, k, pend, H, RH, low4, edges, sv, fill, vfill, lane, below_me, cardS, best,
                                ccp);
        }
        if (fill != 0u) {
            const uint2 e = lane < fill ? sv[lane] : make_uint2(0u, 0u);
            wave_sync_lds();
            push_valid<CM>(L, M, S, A, k, e, lane < fill && ccp_lb(L, e.x, e.y), sv + kSurvCap, vfill, lane,
                           below_me, cardS, best, ccp);
        }
        if (vfill != 0u) {
            const uint2 e = lane < vfill ? sv[kSurvCap + lane] : make_uint2(0u, 0u);
            wave_sync_lds();
            if (lane < vfill) eval_lb<CM>(L, M, S, A, k, e.x, e.y, cardS, best, ccp);
        }
    }
}


// True if the connected set S induces a tree (|S| - 1 edges).
__device__ __forceinline__ bool induces_tree(const LdsGraph &L, uint32_t S) {
    uint32_t e2 = 0;
    for (uint32_t T = S; T; T &= T - 1) e2 += (uint32_t)popc32(L.adj[ctz32(T)] & S);
    return e2 == 2u * (uint32_t)(popc32(S) - 1);
}

// Alg. 2 on one connected S whose induced subgraph is a tree, one lane per
// set: every edge (u, v) of G[S] with u < v gives the pair
// (grow({u}, S - {v}), the rest), both orientations costed.  The memo
// gathers of kB pairs are issued before any of them is used.
template <int CM>
__device__ __forceinline__ void eval_treelike_set(const LdsGraph &L, const MemoPtrs &M, uint32_t S,
                                                  unsigned long long &ccp) {
    constexpr int kB = 4;
    const int k = popc32(S);
    const double cardS = card_of(L, S);
    Key best = worst_key();
    uint32_t V = S, U = 0, vbit = 0;
    while (V | U) {
        uint32_t Av[kB];
        uint64_t ia[kB], ib[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            Av[b] = 0;
            ia[b] = 0;
            ib[b] = 0;
            while (!U && V) {
                vbit = lowbit(V);
                V ^= vbit;
                U = L.adj[ctz32(vbit)] & S & (vbit - 1u);
            }
            if (U) {
                const uint32_t ubit = lowbit(U);
                U ^= ubit;
                const uint32_t A = grow(L.nb, ubit, S & ~vbit);
                uint32_t ra, rb;
                split_ranks(L, S, A, ra, rb);
                const int ka = popc32(A);
                Av[b] = A;
                ia[b] = L.loff[ka] + ra;
                ib[b] = L.loff[k - ka] + rb;
            }
        }
        double cA[kB], cB[kB], kA[kB], kB2[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            cA[b] = cB[b] = kA[b] = kB2[b] = 0.0;
            if (!Av[b]) continue;
            cA[b] = M.cost[ia[b]];
            cB[b] = M.cost[ib[b]];
            if (CM != MPDP_COST_COUT) {
                kA[b] = M.card[ia[b]];
                kB2[b] = M.card[ib[b]];
            }
        }
#pragma unroll
        for (int b = 0; b < kB; ++b)
            if (Av[b]) eval_vals<CM>(Av[b], S ^ Av[b], cA[b], cB[b], kA[b], kB2[b], cardS, best);
    }
    ccp += (unsigned long long)(k - 1);
    store_best(M, memo_index(L, S), best, cardS);
}




// One wave's share of a depth-one tree level (see eval_flat_sets).  The
// connected sets of k relations are {0} + T for the (k - 1)-subsets T of
// relations 1 .. n - 1, so the wave walks the colex ranks of T' = T >> 1
// among the (k - 1)-subsets of n - 1 relations: every rank is a connected
// set, with nothing to filter.  Every set of a level costs the same.  Of
// the ranks [lo, lo + len) that its group of `waves` waves shares, a wave
// takes the blocks of 64 * kTreeChunk ranks round-robin for as many full
// rounds as fit (so that, at any time, the group works on one window of the
// level and its gathers share the caches), then an equal part of what
// remains, so that no wave idles while others finish a last block.  In a
// block each lane unranks kTreeChunk consecutive ranks
// (the first, then same-popcount successors) into the wave's LDS block, and
// then evaluates the ranks lane, 64 + lane, ..., R at a time, so that
// neighbouring lanes cost neighbouring sets (their gathers and stores share
// lines).  The block has one pad word per 8, which keeps both the writes
// (stride kTreeChunk) and the reads (stride 1) free of bank conflicts.  In
// the last, partial block a group of R slots that is full on every lane
// still goes R at a time; only the group that straddles the end goes one
// slot at a time.  Pascal's rule C(t + 1, j + 1) = C(t, j + 1) + C(t, j)
// gives the sum eval_flat_sets takes, bsum(S) = C(0, 0) +
// sum_j C(t'_j + 1, j + 1) = 1 + rank(T') + bsum(T').
constexpr __host__ __device__ int flat_block_words(int chunk) { return 64 * chunk + 64 * chunk / 8; }

template <int CM, int kTreeChunk, int R>
__device__ void level_flat_wave(const LdsGraph &L, const MemoPtrs &M, int n, uint32_t k, uint64_t lo, uint64_t len,
                                uint64_t wave, uint64_t waves, uint32_t *blk_set, uint32_t *blk_bsum, uint32_t lane) {
    static_assert(kTreeChunk % R == 0, "sets per lane come in groups of R");
    const uint64_t per_wave = 64ull * kTreeChunk;
    const uint64_t off_k = L.loff[k], off_km1 = L.loff[k - 1];
    const double *cost_km1 = M.cost + off_km1;
    const double *card_km1 = M.card + off_km1;
    const uint64_t rounds = len / (waves * per_wave);
    const uint64_t tail_lo = lo + rounds * waves * per_wave, tail_len = lo + len - tail_lo;
    for (uint64_t it = 0; it <= rounds; ++it) {
        uint64_t base, r_end;
        if (it < rounds) {
            base = lo + (it * waves + wave) * per_wave;
            r_end = base + per_wave;
        } else {
            base = tail_lo + tail_len * wave / waves;
            r_end = tail_lo + tail_len * (wave + 1) / waves;
            if (base >= r_end) break;
        }
        const uint64_t r0 = base + (uint64_t)lane * kTreeChunk;
        uint32_t bT = 0;
        uint32_t Tp = r0 < r_end ? colex_unrank_b(L.binom, n - 1, (int)k - 1, (uint32_t)r0, bT) : 0u;
#pragma unroll
        for (int j = 0; j < kTreeChunk; ++j) {
            const uint32_t e = lane * kTreeChunk + (uint32_t)j;  // element of the block
            blk_set[e + e / 8] = (Tp << 1) | 1u;
            blk_bsum[e + e / 8] = 1u + (uint32_t)(r0 + (uint64_t)j) + bT;
            if (r0 + (uint64_t)j + 1 < r_end) {
                bT = next_bsum(Tp, bT);
                Tp = next_subset(Tp);
            }
        }
        wave_sync_lds();
        const uint64_t left = r_end - base;  // elements of this block in range (uniform)
#pragma unroll
        for (int j = 0; j < kTreeChunk; j += R) {
            if ((uint64_t)(j + R) * 64u <= left) {  // the whole group, on every lane
                uint32_t s[R], b[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t e = (uint32_t)(j + r) * 64u + lane;
                    s[r] = blk_set[e + e / 8];
                    b[r] = blk_bsum[e + e / 8];
                }
                eval_flat_sets<CM, R>(L, M, s, b, k, off_k, cost_km1, card_km1);
            } else if ((uint64_t)j * 64u < left) {  // the group that straddles the end
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t e = (uint32_t)(j + r) * 64u + lane;
                    if (e < left) {
                        const uint32_t s1 = blk_set[e + e / 8], b1 = blk_bsum[e + e / 8];
                        eval_flat_sets<CM, 1>(L, M, &s1, &b1, k, off_k, cost_km1, card_km1);
                    }
                }
            }
        }
        wave_sync_lds();
    }
}

// One wave's share of an Alg. 2 level (unrank, filter, evaluate, prune and
// scatter fused): it walks the ranges w0, w0 + wstride, ... (below wend) of
// 64 * kTreeChunk colex ranks (kTreeChunk consecutive ranks per lane: unrank the
// first, then the same-popcount successor), appends the connected sets to
// its LDS ring (kRingN entries) in rank order, each with its sum of
// C(s_i, i), and evaluates 64 * kTreeSetsPerLane of them at a time,
// kTreeSetsPerLane per lane, so no lane idles on a disconnected candidate.
// Returns the number of connected sets it found (uniform across the wave).
// Outputs of the unfused-prune ablation (see TreeSink): the pair keys, the
// set records and the counter that hands out their slots.
struct UnfusedOut {
    PairKey *keys;
    PruneRec *recs;
    uint32_t *slots;
};

// Slots for `count` sets (the lanes below count), one atomic per wave.
__device__ __forceinline__ uint32_t take_slots(uint32_t *slots, uint32_t count, uint32_t lane) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(slots, count);
    return (uint32_t)__shfl((int)base, 0) + lane;
}

template <int CM, int kTreeChunk, bool kCompact = true, int kRingN = kRing, int kTreeSetsPerLane = 1,
          int kPairBatch = MPDP_TREE_PAIR_BATCH, bool kUnfused = false, bool kFlat = false,
          bool kBatchKeys = false>
__device__ uint32_t level_tree_wave(const LdsGraph &L, const MemoPtrs &M, int n, uint32_t k, uint64_t ncand,
                                    uint64_t w0, uint64_t wstride, uint64_t wend, uint32_t *ring,
                                    uint32_t *ring_bsum, uint32_t lane,
                                    UnfusedOut uo = UnfusedOut{nullptr, nullptr, nullptr}) {
    static_assert(kRingN >= 64 * kTreeSetsPerLane - 1 + 64 * kTreeChunk, "ring too small");
    static_assert(!kUnfused || (kCompact && kTreeSetsPerLane == 1), "the unfused ablation is one set per lane");
    TreeSink sink;
    sink.keys = uo.keys;
    sink.recs = uo.recs;
    const unsigned long long below_me = (1ull << lane) - 1ull;
    const uint64_t per_wave = 64ull * kTreeChunk;
    const uint64_t off_k = L.loff[k], off_km1 = L.loff[k - 1];
    const double *cost_km1 = M.cost + off_km1;
    const double *card_km1 = M.card + off_km1;
    uint32_t head = 0, tail = 0;  // ring cursors, uniform across the wave
    for (uint64_t w = w0; w < wend; w += wstride) {
        const uint64_t r0 = w * per_wave + (uint64_t)lane * kTreeChunk;
        uint32_t b = 0;
        uint32_t S = r0 < ncand ? colex_unrank_b(L.binom, n, (int)k, (uint32_t)r0, b) : 0u;
        uint32_t sets[kTreeChunk], bsums[kTreeChunk];
        uint32_t keep = 0;
#pragma unroll
        for (int j = 0; j < kTreeChunk; ++j) {
            sets[j] = S;
            bsums[j] = b;
            if (r0 + (uint64_t)j < ncand) {
                // G[S] is a forest whose edges are the members with their
                // parent in S; it is one tree when there are k - 1 of them
                if ((uint32_t)popc32(S & children(L.ch, S)) == k - 1) keep |= 1u << j;
                b = next_bsum(S, b);
                S = next_subset(S);
            }
        }
        const uint32_t mine = (uint32_t)popc32(keep);
        // exclusive prefix of `mine` (at most kTreeChunk) across the wave,
        // one ballot per bit of kTreeChunk
        constexpr int kBits = kTreeChunk >= 8 ? 4 : (kTreeChunk >= 4 ? 3 : (kTreeChunk >= 2 ? 2 : 1));
        static_assert(kTreeChunk < (1 << kBits), "prefix bits");
        uint32_t before = 0;
#pragma unroll
        for (int b = 0; b < kBits; ++b)
            before += (uint32_t)__popcll(__ballot((mine >> b) & 1u) & below_me) << b;
        const uint32_t total = (uint32_t)__shfl((int)(before + mine), 63);
        if (!kCompact) {  // ablation: each lane evaluates the sets it kept, lanes diverge
#pragma unroll
            for (int j = 0; j < kTreeChunk; ++j)
                if (keep & (1u << j)) {
                    if constexpr (kFlat)
                        eval_flat_sets<CM, 1, kPairBatch>(L, M, &sets[j], &bsums[j], k, off_k, cost_km1, card_km1);
                    else
                        eval_tree_set<CM, kPairBatch>(L, M, sets[j], bsums[j], k, off_k, cost_km1, card_km1);
                }
            tail += total;
            head = tail;
            continue;
        }
        uint32_t pos = tail + before;
#pragma unroll
        for (int j = 0; j < kTreeChunk; ++j)
            if (keep & (1u << j)) {
                ring[pos % kRingN] = sets[j];
                ring_bsum[pos % kRingN] = bsums[j];
                ++pos;
            }
        tail += total;
        wave_sync_lds();
        while (tail - head >= 64u * kTreeSetsPerLane) {
            uint32_t s[kTreeSetsPerLane], r[kTreeSetsPerLane];
#pragma unroll
            for (int j = 0; j < kTreeSetsPerLane; ++j) {
                s[j] = ring[(head + 64u * j + lane) % kRingN];
                r[j] = ring_bsum[(head + 64u * j + lane) % kRingN];
            }
            if (kUnfused) sink.slot[0] = take_slots(uo.slots, 64u, lane);
            if constexpr (kFlat)
                eval_flat_sets<CM, kTreeSetsPerLane, kPairBatch, kUnfused>(L, M, s, r, k, off_k, cost_km1, card_km1,
                                                                           sink);
            else
                eval_tree_sets<CM, kTreeSetsPerLane, kPairBatch, kUnfused, kBatchKeys>(L, M, s, r, k, off_k, cost_km1,
                                                                                       card_km1, sink);
            head += 64u * kTreeSetsPerLane;
        }
        wave_sync_lds();
    }
    while (tail - head >= 64) {
        const uint32_t s = ring[(head + lane) % kRingN], r = ring_bsum[(head + lane) % kRingN];
        if (kUnfused) sink.slot[0] = take_slots(uo.slots, 64u, lane);
        if constexpr (kFlat)
            eval_flat_sets<CM, 1, kPairBatch, kUnfused>(L, M, &s, &r, k, off_k, cost_km1, card_km1, sink);
        else
            eval_tree_sets<CM, 1, kPairBatch, kUnfused, kBatchKeys>(L, M, &s, &r, k, off_k, cost_km1, card_km1, sink);
        head += 64;
    }
    if (tail != head) {
        if (kUnfused) sink.slot[0] = take_slots(uo.slots, tail - head, lane);
        if (lane < tail - head) {
            const uint32_t s = ring[(head + lane) % kRingN], r = ring_bsum[(head + lane) % kRingN];
            if constexpr (kFlat)
                eval_flat_sets<CM, 1, kPairBatch, kUnfused>(L, M, &s, &r, k, off_k, cost_km1, card_km1, sink);
            else
                eval_tree_sets<CM, 1, kPairBatch, kUnfused, kBatchKeys>(L, M, &s, &r, k, off_k, cost_km1, card_km1,
                                                                        sink);
        }
    }
    wave_sync_lds();
    return tail;
}

// A small Alg. 2 level: groups of P lanes take one colex rank each (ranks
// w * (64 / P) + group for w = w0, w0 + wstride, ... below wend); a group
// whose candidate induces a tree costs it with eval_tree_set_split.  Lanes
// of a group unrank and test the same candidate, so groups never diverge
// inside.  Returns the number of connected sets it found (uniform across
// the wave).
template <int CM, int P>
__device__ uint32_t level_tree_split_wave(const LdsGraph &L, const MemoPtrs &M, int n, uint32_t k, uint64_t ncand,
                                          uint64_t w0, uint64_t wstride, uint64_t wend, uint32_t lane) {
    constexpr uint32_t kGroups = 64 / P;
    const uint32_t group = lane / P, sub = lane % P;
    const uint64_t off_k = L.loff[k], off_km1 = L.loff[k - 1];
    const double *cost_km1 = M.cost + off_km1;
    const double *card_km1 = M.card + off_km1;
    uint32_t found = 0;
    for (uint64_t w = w0; w < wend; w += wstride) {
        const uint64_t r = w * kGroups + group;
        const uint32_t S = r < ncand ? colex_unrank(L.binom, n, (int)k, (uint32_t)r) : 0u;
        const bool tree = r < ncand && (uint32_t)popc32(S & children(L.ch, S)) == k - 1;
        found += (uint32_t)__popcll(__ballot(tree && sub == 0));
        if (tree) eval_tree_set_split<CM, P>(L, M, S, (uint32_t)r, k, sub, off_k, cost_km1, card_km1);
    }
    return found;
}

// One wave's share of the unrank + filter step for the block-based path:
// kFilterChunk consecutive colex ranks per lane.  The connected sets that
// induce a tree are appended at the front of `list` (count in *ntree), the
// others at its back, from list[cap - 1] downwards (count in *ngen); each
// lane's counts are prefixed across the wave with one ballot per count bit
// and one atomic per list and wave (global or LDS) reserves the range.
__device__ void filter_wave(const LdsGraph &L, int n, uint32_t k, uint64_t ncand, uint64_t w0, uint64_t wstride,
                            uint32_t *list, uint32_t cap, uint32_t *ntree, uint32_t *ngen, uint32_t lane,
                            bool split = true) {
    const unsigned long long below_me = (1ull << lane) - 1ull;
    const uint64_t per_wave = 64ull * kFilterChunk;
    for (uint64_t w = w0; w * per_wave < ncand; w += wstride) {
        const uint64_t r0 = w * per_wave + (uint64_t)lane * kFilterChunk;
        uint32_t S = r0 < ncand ? colex_unrank(L.binom, n, (int)k, (uint32_t)r0) : 0u;
        uint32_t sets[kFilterChunk];
        uint32_t keep_t = 0, keep_g = 0;
#pragma unroll
        for (int j = 0; j < kFilterChunk; ++j) {
            sets[j] = S;
            if (r0 + (uint64_t)j < ncand) {
                if (grow(L.nb, lowbit(S), S) == S) {
                    if (split && induces_tree(L, S)) keep_t |= 1u << j;
                    else keep_g |= 1u << j;
                }
                S = next_subset(S);
            }
        }
        const uint32_t mt = (uint32_t)popc32(keep_t), mg = (uint32_t)popc32(keep_g);
        uint32_t bt = 0, bg = 0;
#pragma unroll
        for (int b = 0; b < 5; ++b) {  // exclusive prefixes (counts <= 16) across the wave
            bt += (uint32_t)__popcll(__ballot((mt >> b) & 1u) & below_me) << b;
            bg += (uint32_t)__popcll(__ballot((mg >> b) & 1u) & below_me) << b;
        }
        const uint32_t tot_t = (uint32_t)__shfl((int)(bt + mt), 63);
        const uint32_t tot_g = (uint32_t)__shfl((int)(bg + mg), 63);
        if (tot_t) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(ntree, tot_t);
            base = (uint32_t)__shfl((int)base, 0) + bt;
#pragma unroll
            for (int j = 0; j < kFilterChunk; ++j)
                if (keep_t & (1u << j)) list[base++] = sets[j];
        }
        if (tot_g) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(ngen, tot_g);
            base = (uint32_t)__shfl((int)base, 0) + bg;
#pragma unroll
            for (int j = 0; j < kFilterChunk; ++j)
                if (keep_g & (1u << j)) list[cap - 1u - base++] = sets[j];
        }
    }
}

// One wave's share of the light work of a block-based level.  Work item i
// (i = w0, w0 + wstride, ...) is either a group of 64 tree-inducing sets
// from the front of `list`, one per lane (Alg. 2 on G[S]), or, past the
// groups, one other set from the back of `list`, taken by the whole wave
// (Alg. 3 over its blocks).  A set with more than kHeavyChunks 16-candidate
// chunks is appended to `heavy` for a whole workgroup instead.
template <int CM, bool kChunkTables = true>
__device__ void light_sets(const LdsGraph &L, const MemoPtrs &M, const uint32_t *list, uint32_t cap, uint32_t ntree,
                           uint32_t ngen, uint32_t w0, uint32_t wstride, WaveScratch &W, uint32_t *heavy,
                           uint32_t *nheavy, uint32_t lane, unsigned long long &ccp, unsigned long long &evaluated,
                           bool dpsub = false, uint32_t heavy_chunks = kHeavyChunks, uint2 *sv = nullptr) {
    const uint32_t groups = (ntree + 63u) >> 6;
    for (uint32_t i = w0; i < groups + ngen; i += wstride) {
        if (i < groups) {
            const uint32_t idx = (i << 6) + lane;
            if (idx < ntree) {
                const uint32_t S = list[idx];
                eval_treelike_set<CM>(L, M, S, ccp);
                evaluated += 2ull * (unsigned long long)(popc32(S) - 1);
            }
            continue;
        }
        const uint32_t S = list[cap - 1u - (i - groups)];
        const SetBlocks sb = dpsub ? whole_set(S, W, (int)lane, 64u) : analyze_set(L, S, W, (int)lane, 64u);
        if ((kChunkTables ? sb.work16 : sb.chunks16) > heavy_chunks) {
            if (lane == 0) heavy[atomicAdd(nheavy, 1u)] = S;
            wave_sync_lds();
            continue;
        }
        if (lane == 0) evaluated += sb.evaluated;
        wave_sync_lds();
        const double cardS = card_of_wave(L, S, lane);
        Key best = worst_key();
        eval_chunks<CM, kChunkTables>(L, M, W, S, sb, lane, 64u, cardS, best, ccp, sv);
        best = wave_min(best);
        const uint64_t at = memo_index_wave(L, S, lane);
        if (lane == 0) store_best(M, at, best, cardS);
        wave_sync_lds();
    }
}

// Plan extraction scratch (LDS) and routine.  Join nodes are numbered in
// post-order (left subtree, right subtree, node), after the n relations.  A
// node whose subtree covers S and starts after `start` finished join nodes
// gets number n + start + |S| - 2; its left child L starts at `start`, its
// right child at start + |L| - 1.  So numbers follow from set sizes alone
// and wave 0 can walk the plan tree top-down one depth per round, every
// node of the frontier reading its left set at once (the only dependent
// chain is the tree's depth); then all `nthreads` threads fill cost, card
// and operator of every node.  Memo indices are summed by the wave, one
// member per lane, one frontier set at a time, and kept for the fill.
// Returns false if the memo is inconsistent.
struct PlanScratch {
    uint64_t node_at[64];
    uint32_t node_set[64];
    int node_l[64], node_r[64];
    uint32_t fr_set[2][32];
    int fr_start[2][32];
    int error;
};

// Memo index of S from binom and loff alone, summed over the wave (every
// lane active): lane v < 32 adds the term of relation v.
__device__ __forceinline__ uint64_t memo_index_wave_t(const uint32_t *binom, const uint64_t *loff, uint32_t S,
                                                      uint32_t lane) {
    uint32_t term = 0;
    if (lane < 32 && ((S >> lane) & 1u)) term = binom[lane * 33 + popc32(S & ((1u << lane) - 1u)) + 1];
    return loff[popc32(S)] + wave_sum32(term);
}

__device__ bool extract_plan(const uint32_t *binom, const uint64_t *loff, const MemoPtrs &M, uint32_t n,
                             mpdp_plan_node *plan, double *root_cost, PlanScratch &P, uint32_t t,
                             uint32_t nthreads) {
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    if (t < 64) {
        const uint32_t lane = t;
        const unsigned long long below_me = (1ull << lane) - 1ull;
        if (lane == 0) {
            P.error = 0;
            P.fr_set[0][0] = full;
            P.fr_start[0][0] = 0;
        }
        wave_sync_lds();
        // the root's cost is read while the walk goes on
        const uint64_t root_at = memo_index_wave_t(binom, loff, full, lane);
        const double root_c = lane == 0 ? M.cost[root_at] : 0.0;
        int cur = 0;
        uint32_t nfr = n > 1 ? 1u : 0u;  // frontier size, uniform; at most 31 join nodes per depth
        bool bad = false;
        for (uint32_t depth = 0; nfr != 0 && depth < n; ++depth) {
            uint64_t my_at = 0;  // lane j: index of frontier set j
            for (uint32_t j = 0; j < nfr; ++j) {
                const uint64_t at = memo_index_wave_t(binom, loff, P.fr_set[cur][j], lane);
                if (lane == j) my_at = at;
            }
            uint32_t push = 0, c0 = 0, c1 = 0;  // join children to visit next: c0, then c1
            int s0 = 0, s1 = 0;
            if (lane < nfr) {
                const uint32_t S = P.fr_set[cur][lane];
                const int st = P.fr_start[cur][lane];
                const uint32_t Lft = M.left[my_at];
                if (Lft == 0 || (Lft & ~S) != 0 || Lft == S) {
                    bad = true;
                } else {
                    const uint32_t Rgt = S & ~Lft;
                    const int nl = popc32(Lft), nr = popc32(Rgt);
                    const int rst = st + nl - 1;
                    const int idx = (int)n + st + popc32(S) - 2;
                    P.node_set[idx] = S;
                    P.node_at[idx] = my_at;
                    P.node_l[idx] = nl >= 2 ? (int)n + st + nl - 2 : ctz32(Lft);
                    P.node_r[idx] = nr >= 2 ? (int)n + rst + nr - 2 : ctz32(Rgt);
                    if (nl >= 2) { c0 = Lft; s0 = st; push = 1; }
                    if (nr >= 2) {
                        if (push) { c1 = Rgt; s1 = rst; push = 2; }
                        else { c0 = Rgt; s0 = rst; push = 1; }
                    }
                }
            }
            // exclusive prefix of `push` (<= 2) across the wave
            const uint32_t before = (uint32_t)__popcll(__ballot(push & 1u) & below_me) +
                                    2u * (uint32_t)__popcll(__ballot((push >> 1) & 1u) & below_me);
            const uint32_t total = (uint32_t)__shfl((int)(before + push), 63);
            const int nxt = cur ^ 1;
            if (push >= 1 && before < 32) {
                P.fr_set[nxt][before] = c0;
                P.fr_start[nxt][before] = s0;
            }
            if (push >= 2 && before + 1 < 32) {
                P.fr_set[nxt][before + 1] = c1;
                P.fr_start[nxt][before + 1] = s1;
            }
            if (total > 32) bad = true;
            wave_sync_lds();
            nfr = total > 32 ? 0u : total;
            cur = nxt;
        }
        if (nfr != 0) bad = true;
        if (__ballot(bad) != 0ull && lane == 0) P.error = 1;
        if (lane == 0) *root_cost = root_c;
    }
    __syncthreads();
    if (P.error) return false;
    for (uint32_t v = t; v < n; v += nthreads) {
        const uint64_t at = loff[1] + v;
        plan[v] = mpdp_plan_node{-1, -1, 1u << v, MPDP_OP_SCAN, M.cost[at], M.card[at]};
    }
    for (uint32_t j = n + t; j + 1 < 2 * n; j += nthreads) {
        const uint64_t at = P.node_at[j];
        plan[j] = mpdp_plan_node{P.node_l[j], P.node_r[j], P.node_set[j], (uint32_t)M.op[at], M.cost[at], M.card[at]};
    }
    return true;
}

}  // namespace
}  // namespace mpdp
