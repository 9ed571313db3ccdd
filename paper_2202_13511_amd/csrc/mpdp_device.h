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
constexpr int kTreeChunkMax = 4;    // consecutive ranks per lane in k_level_tree (1, 2 or 4)
constexpr int kRing = 384;          // per-wave ring of connected sets (>= 63 + 64 * kTreeChunkMax)
constexpr uint32_t kPersistGrid = 1024;  // workgroups that keep the whole chip busy (4 per CU)
constexpr int kEvalChunk = 16;      // block-local candidates per lane chunk
constexpr uint32_t kHeavyChunks = 256;   // above this many chunks a set goes to k_eval_heavy
constexpr int kHeavyBlock = 1024;        // threads per heavy set
constexpr uint32_t kMaxGrid = 8192; // workgroups per launch (grid-stride beyond)

static_assert(kRing >= 63 + 64 * kTreeChunkMax, "ring too small");

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

// Memo index of T: level offset plus colex rank.
__device__ __forceinline__ uint64_t memo_index(const LdsGraph &L, uint32_t T) {
    uint32_t r = 0;
    int i = 1;
    for (uint32_t U = T; U; U &= U - 1, ++i) r += L.binom[ctz32(U) * 33 + i];
    return L.loff[i - 1] + r;
}

// Colex unrank of rank r among the k-subsets of n relations.
__device__ __forceinline__ uint32_t colex_unrank(const uint32_t *binom, int n, int k, uint32_t r) {
    uint32_t S = 0;
    int c = n - 1;
    for (int i = k; i >= 1; --i) {
        while (binom[c * 33 + i] > r) --c;
        r -= binom[c * 33 + i];
        S |= 1u << c;
        --c;
    }
    return S;
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


// Alg. 2 for one connected S of a tree join graph.  With the tree rooted at
// relation 0, removing the edge (parent(c), c) of G[S] gives the pair
// (desc(c) & S, S minus that) for every c in S whose parent is in S.
// When desc(c) & S = {c} the complement's colex rank follows from prefix
// sums, rank(S - s_j) = sum_{i<j} C(s_i, i+1) + sum_{i>j} C(s_i, i), and the
// singleton's cost and card come from LDS.  Pairs are taken in batches of
// kPairBatch whose memo gathers are all issued before any is used; the batch
// keeps 32-bit ranks only, so that eight waves fit on a SIMD.
template <int CM>
__device__ __forceinline__ void eval_tree_set(const LdsGraph &L, const MemoPtrs &M, uint32_t S, uint64_t off_k,
                                              const double *__restrict__ cost_km1,
                                              const double *__restrict__ card_km1) {
    constexpr int kPairBatch = (CM == MPDP_COST_COUT) ? 8 : 4;
    uint32_t rank = 0, bsum = 0;
    {
        int i = 0;
        for (uint32_t T = S; T; T &= T - 1, ++i) {
            const int v = ctz32(T);
            rank += L.binom[v * 33 + i + 1];
            bsum += L.binom[v * 33 + i];
        }
    }
    const double cardS = card_of(L, S);
    Key best = worst_key();
    uint32_t pa = 0, pb = 0, T = S;
    int i = 0;
    while (T) {
        uint32_t Av[kPairBatch], rk[kPairBatch];
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            Av[u] = 0;
            rk[u] = 0;
            while (T) {
                const int c = ctz32(T);
                T &= T - 1;
                const uint32_t a_i = L.binom[c * 33 + i + 1];
                pb += L.binom[c * 33 + i];
                ++i;
                const bool take = (S & L.pbit[c]) != 0;
                if (take) {
                    Av[u] = L.desc[c] & S;
                    rk[u] = pa + (bsum - pb);  // colex rank of S - {c}
                }
                pa += a_i;
                if (take) break;
            }
        }
        double cA[kPairBatch], cB[kPairBatch], kA[kPairBatch], kB[kPairBatch];
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            const uint32_t A = Av[u];
            if (!A) continue;
            if ((A & (A - 1)) == 0) {
                cB[u] = cost_km1[rk[u]];
                if (CM != MPDP_COST_COUT) kB[u] = card_km1[rk[u]];
                const int c = ctz32(A);
                cA[u] = L.bcost[c];
                kA[u] = L.card[c];
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
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u)
            if (Av[u]) eval_vals<CM>(Av[u], S ^ Av[u], cA[u], cB[u], kA[u], kB[u], cardS, best);
    }
    store_best(M, off_k + rank, best, cardS);
}


// Key reduction across the 64 lanes of a wave.
__device__ __forceinline__ Key wave_min(Key b) {
    for (int off = 32; off >= 1; off >>= 1) {
        Key o;
        o.c = (unsigned long long)__shfl_xor((long long)b.c, off);
        o.l = (uint32_t)__shfl_xor((int)b.l, off);
        o.op = (uint32_t)__shfl_xor((int)b.op, off);
        if (key_less(o, b)) b = o;
    }
    return b;
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
    uint32_t total_chunks;  // candidate chunks over all blocks
    unsigned long long evaluated;  // Alg. 3 candidates of S: sum over blocks of 2^b - 2
};

// Blocks of G[S] for one connected S, computed by one wave:
//  1. cut vertices: lane v checks whether G[S - v] is connected;
//  2. split S at a cut vertex into pieces {x} + component, and split pieces
//     again until a piece has no cut vertex of its own.  A piece is a union
//     of blocks of S; its attachment set holds the split vertices it still
//     contains, which are not cut vertices of the piece, while every other
//     cut vertex of S inside the piece is.  Control flow is uniform; the
//     piece stack lives one entry per lane.
// The block list, completeness flags and candidate-chunk prefix go to W.
__device__ SetBlocks analyze_set(const LdsGraph &L, uint32_t S, WaveScratch &W, int lane) {
    // degrees in G[S]; a connected S with |S| - 1 edges induces a tree, whose
    // blocks are its edges and whose cut vertices are its inner relations
    const bool mine = lane < 32 && ((S >> lane) & 1u);
    const uint32_t deg = mine ? (uint32_t)popc32(L.adj[lane] & S) : 0u;
    uint32_t edges2 = deg;
    for (int off = 32; off >= 1; off >>= 1) edges2 += (uint32_t)__shfl_xor((int)edges2, off);
    const int kS = popc32(S);
    if (edges2 == 2u * (uint32_t)(kS - 1)) {
        const uint32_t A = (uint32_t)__ballot(mine && deg >= 2);
        // lane v owns the edges to its smaller neighbours in S
        const uint32_t lower = mine ? (L.adj[lane] & S & ((1u << lane) - 1u)) : 0u;
        const uint32_t cnt = (uint32_t)popc32(lower);
        uint32_t before = 0;
        for (int b = 0; b < 5; ++b)
            before += (uint32_t)__popcll(__ballot((cnt >> b) & 1u) & ((1ull << lane) - 1ull)) << b;
        uint32_t at = before;
        for (uint32_t U = lower; U; U &= U - 1, ++at) {
            W.blk[at] = lowbit(U) | (1u << lane);
            W.full[at] = 1;
            W.cpre[at] = at;
        }
        if (lane == 0) W.cpre[kS - 1] = (uint32_t)(kS - 1);
        return SetBlocks{A, (uint32_t)(kS - 1), 2ull * (unsigned long long)(kS - 1)};
    }

    bool cut = false;
    if (mine) {
        const uint32_t R = S & ~(1u << lane);
        cut = grow(L.nb, lowbit(R), R) != R;
    }
    const uint32_t A = (uint32_t)__ballot(cut);

    uint32_t stkP = 0, stkA = 0, myblk = 0;
    int sp = 0, nblk = 0, steps = 0;
    if (lane == 0) { stkP = S; stkA = 0; }
    sp = 1;
    while (sp > 0 && steps < 2 * kMaxRel) {
        ++steps;
        --sp;
        const uint32_t P = rdlane(stkP, sp);
        const uint32_t at = rdlane(stkA, sp);
        const uint32_t cuts = A & P & ~at;
        if (cuts == 0) {
            if (lane == nblk) myblk = P;
            nblk += nblk < kMaxRel - 1 ? 1 : 0;
            continue;
        }
        const uint32_t x = lowbit(cuts);
        uint32_t rem = P & ~x;
        while (rem) {
            const uint32_t K = grow(L.nb, lowbit(rem), rem);
            rem &= ~K;
            if (lane == sp) { stkP = K | x; stkA = (at | x) & (K | x); }
            sp += sp < 63 ? 1 : 0;
        }
    }

    // per-block candidate counts (lane i owns block i)
    uint32_t chunks = 0, complete = 0;
    if (lane < nblk) {
        const int bs = popc32(myblk);
        const uint32_t half = (1u << (bs - 1)) - 1u;
        chunks = (half + kEvalChunk - 1) / kEvalChunk;
        uint32_t deg = 0;
        for (uint32_t T = myblk; T; T &= T - 1) deg += popc32(L.adj[ctz32(T)] & myblk);
        complete = deg == (uint32_t)(bs * (bs - 1));
    }
    uint32_t acc = 0, mypre = 0;
    unsigned long long evaluated = 0;
    for (int i = 0; i < nblk; ++i) {
        const uint32_t c = rdlane(chunks, i);
        if (lane == i) mypre = acc;
        acc += c;
        evaluated += (1ull << popc32(rdlane(myblk, i))) - 2ull;
    }
    if (lane < nblk) { W.blk[lane] = myblk; W.full[lane] = complete; W.cpre[lane] = mypre; }
    if (lane == 0) W.cpre[nblk] = acc;
    return SetBlocks{A, acc, evaluated};
}

// Colex ranks of Sl and of S - Sl in one pass over the members of S.
__device__ __forceinline__ void split_ranks(const LdsGraph &L, uint32_t S, uint32_t Sl, uint32_t &rl, uint32_t &rr) {
    uint32_t a = 0, b = 0;
    int il = 1, ir = 1;
    for (uint32_t T = S; T; T &= T - 1) {
        const int v = ctz32(T);
        if ((Sl >> v) & 1u) a += L.binom[v * 33 + il++];
        else b += L.binom[v * 33 + ir++];
    }
    rl = a;
    rr = b;
}

// Alg. 3 candidates of the chunks ch = first, first + stride, ... of S: for
// each block-local lb holding the block's lowest relation (lb != block, so
// each unordered pair is met once and both orientations are costed) the CCP
// check is that G[lb] and G[rb] are connected (they are adjacent because the
// block is); then S_left = grow(lb, S - rb) and S_right = S - S_left.
template <int CM>
__device__ __forceinline__ void eval_chunks(const LdsGraph &L, const MemoPtrs &M, const WaveScratch &W, uint32_t S,
                                            uint32_t A, uint32_t total_chunks, uint32_t first, uint32_t stride,
                                            double cardS, Key &best, unsigned long long &ccp) {
    const int k = popc32(S);
    for (uint32_t ch = first; ch < total_chunks; ch += stride) {
        int bi = 0;
        while (W.cpre[bi + 1] <= ch) ++bi;
        const uint32_t b = W.blk[bi];
        const bool full = W.full[bi] != 0;
        const uint32_t lo = lowbit(b), rest = b ^ lo;
        const uint32_t hb = (1u << (popc32(b) - 1)) - 1u;
        const uint32_t j0 = (ch - W.cpre[bi]) * kEvalChunk;
        const uint32_t j1 = min(j0 + (uint32_t)kEvalChunk, hb);
        uint32_t sub = deposit(j0, rest);
        for (uint32_t j = j0; j < j1; ++j) {
            const uint32_t lb = lo | sub, rb = b ^ lb;
            sub = (sub - rest) & rest;
            if (!full) {
                if (grow(L.nb, lo, lb) != lb) continue;
                if (grow(L.nb, lowbit(rb), rb) != rb) continue;
            }
            ++ccp;
            const uint32_t Sl = (lb & A) ? grow(L.nb, lb, S & ~rb) : lb;
            uint32_t rl, rr;
            split_ranks(L, S, Sl, rl, rr);
            const int kl = popc32(Sl);
            eval_pair<CM>(M, Sl, S ^ Sl, L.loff[kl] + rl, L.loff[k - kl] + rr, cardS, best);
        }
    }
}


__device__ __forceinline__ uint64_t memo_index_t(const uint32_t *binom, const uint64_t *loff, uint32_t T) {
    uint32_t r = 0;
    int i = 1;
    for (uint32_t U = T; U; U &= U - 1, ++i) r += binom[ctz32(U) * 33 + i];
    return loff[i - 1] + r;
}



// One wave's share of an Alg. 2 level (unrank, filter, evaluate, prune and
// scatter fused): it walks the ranges w0, w0 + wstride, ... of 64 *
// kTreeChunk colex ranks (kTreeChunk consecutive ranks per lane: unrank the
// first, then the same-popcount successor), appends the connected sets to
// its LDS ring in rank order and evaluates 64 of them at a time, one per
// lane, so no lane idles on a disconnected candidate.  Returns the number of
// connected sets it found (uniform across the wave).
template <int CM, int kTreeChunk>
__device__ uint32_t level_tree_wave(const LdsGraph &L, const MemoPtrs &M, int n, uint32_t k, uint64_t ncand,
                                    uint64_t w0, uint64_t wstride, uint32_t *ring, uint32_t lane) {
    static_assert(kRing >= 63 + 64 * kTreeChunk, "ring too small");
    const unsigned long long below_me = (1ull << lane) - 1ull;
    const uint64_t per_wave = 64ull * kTreeChunk;
    const uint64_t off_k = L.loff[k], off_km1 = L.loff[k - 1];
    const double *cost_km1 = M.cost + off_km1;
    const double *card_km1 = M.card + off_km1;
    uint32_t head = 0, tail = 0;  // ring cursors, uniform across the wave
    for (uint64_t w = w0; w * per_wave < ncand; w += wstride) {
        const uint64_t r0 = w * per_wave + (uint64_t)lane * kTreeChunk;
        uint32_t S = r0 < ncand ? colex_unrank(L.binom, n, (int)k, (uint32_t)r0) : 0u;
        uint32_t sets[kTreeChunk];
        uint32_t keep = 0;
#pragma unroll
        for (int j = 0; j < kTreeChunk; ++j) {
            sets[j] = S;
            if (r0 + (uint64_t)j < ncand) {
                if (grow(L.nb, lowbit(S), S) == S) keep |= 1u << j;
                S = next_subset(S);
            }
        }
        const uint32_t mine = (uint32_t)popc32(keep);
        uint32_t before = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b)  // exclusive prefix of `mine` (<= 4) across the wave
            before += (uint32_t)__popcll(__ballot((mine >> b) & 1u) & below_me) << b;
        const uint32_t total = (uint32_t)__shfl((int)(before + mine), 63);
        uint32_t pos = tail + before;
#pragma unroll
        for (int j = 0; j < kTreeChunk; ++j)
            if (keep & (1u << j)) ring[(pos++) % kRing] = sets[j];
        tail += total;
        wave_sync_lds();
        while (tail - head >= 64) {
            const uint32_t s = ring[(head + lane) % kRing];
            eval_tree_set<CM>(L, M, s, off_k, cost_km1, card_km1);
            head += 64;
        }
        wave_sync_lds();
    }
    if (tail != head && lane < tail - head) {
        const uint32_t s = ring[(head + lane) % kRing];
        eval_tree_set<CM>(L, M, s, off_k, cost_km1, card_km1);
    }
    wave_sync_lds();
    return tail;
}

// One wave's share of the unrank + filter step for the block-based path:
// kFilterChunk consecutive colex ranks per lane; the wave compacts its
// connected sets in rank order (each lane's count is prefixed across the
// wave with one ballot per count bit) and one atomic on `count` (global or
// LDS) reserves the output range in `list`.
__device__ void filter_wave(const LdsGraph &L, int n, uint32_t k, uint64_t ncand, uint64_t w0, uint64_t wstride,
                            uint32_t *list, uint32_t *count, uint32_t lane) {
    const unsigned long long below_me = (1ull << lane) - 1ull;
    const uint64_t per_wave = 64ull * kFilterChunk;
    for (uint64_t w = w0; w * per_wave < ncand; w += wstride) {
        const uint64_t r0 = w * per_wave + (uint64_t)lane * kFilterChunk;
        uint32_t S = r0 < ncand ? colex_unrank(L.binom, n, (int)k, (uint32_t)r0) : 0u;
        uint32_t sets[kFilterChunk];
        uint32_t keep = 0;
#pragma unroll
        for (int j = 0; j < kFilterChunk; ++j) {
            sets[j] = S;
            if (r0 + (uint64_t)j < ncand) {
                if (grow(L.nb, lowbit(S), S) == S) keep |= 1u << j;
                S = next_subset(S);
            }
        }
        const uint32_t mine = (uint32_t)popc32(keep);
        uint32_t before = 0;
#pragma unroll
        for (int b = 0; b < 5; ++b)  // exclusive prefix of `mine` (<= 16) across the wave
            before += (uint32_t)__popcll(__ballot((mine >> b) & 1u) & below_me) << b;
        const uint32_t total = (uint32_t)__shfl((int)(before + mine), 63);
        if (total == 0) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(count, total);
        base = (uint32_t)__shfl((int)base, 0) + before;
#pragma unroll
        for (int j = 0; j < kFilterChunk; ++j)
            if (keep & (1u << j)) list[base++] = sets[j];
    }
}

// Plan extraction scratch (LDS) and routine: lane 0 of the calling group
// follows the left pointers from the full set (the only dependent chain,
// n - 1 reads) and records the join nodes in post-order; then `nthreads`
// threads fill cost, card and operator of every node.  Returns false if the
// memo is inconsistent.
struct PlanScratch {
    uint32_t node_set[64];
    int node_l[64], node_r[64];
    int node_count;
};

__device__ bool extract_plan(const uint32_t *binom, const uint64_t *loff, const MemoPtrs &M, uint32_t n,
                             mpdp_plan_node *plan, double *root_cost, PlanScratch &P, uint32_t t,
                             uint32_t nthreads) {
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    if (t == 0) {
        int next = (int)n;
        if (n > 1) {
            struct Frame { uint32_t S; uint32_t L; int stage; int li; };
            Frame st[33];
            int sp = 0, ret = -1, guard = 0;
            st[sp++] = Frame{full, M.left[memo_index_t(binom, loff, full)], 0, -1};
            while (sp > 0 && ++guard < 4 * 64) {
                Frame &f = st[sp - 1];
                const uint32_t Lft = f.L;
                if (Lft == 0 || (Lft & ~f.S) != 0 || Lft == f.S) { next = -1; break; }
                const uint32_t Rgt = f.S & ~Lft;
                if (f.stage == 0) {
                    f.stage = 1;
                    if ((Lft & (Lft - 1)) == 0) ret = ctz32(Lft);
                    else {
                        if (sp >= 33) { next = -1; break; }
                        st[sp++] = Frame{Lft, M.left[memo_index_t(binom, loff, Lft)], 0, -1};
                        continue;
                    }
                }
                if (f.stage == 1) {
                    f.li = ret;
                    f.stage = 2;
                    if ((Rgt & (Rgt - 1)) == 0) ret = ctz32(Rgt);
                    else {
                        if (sp >= 33) { next = -1; break; }
                        st[sp++] = Frame{Rgt, M.left[memo_index_t(binom, loff, Rgt)], 0, -1};
                        continue;
                    }
                }
                if (next >= 63) { next = -1; break; }
                P.node_set[next] = f.S;
                P.node_l[next] = f.li;
                P.node_r[next] = ret;
                ret = next++;
                --sp;
            }
            if (next >= 0 && (sp != 0 || next != (int)(2 * n - 1))) next = -1;
        }
        P.node_count = next;
        *root_cost = M.cost[memo_index_t(binom, loff, full)];
    }
    __syncthreads();
    const int total = P.node_count;
    if (total < 0) return false;
    for (uint32_t v = t; v < n; v += nthreads) {
        const uint64_t at = loff[1] + v;
        plan[v] = mpdp_plan_node{-1, -1, 1u << v, MPDP_OP_SCAN, M.cost[at], M.card[at]};
    }
    for (int j = (int)n + (int)t; j < total; j += (int)nthreads) {
        const uint64_t at = memo_index_t(binom, loff, P.node_set[j]);
        plan[j] = mpdp_plan_node{P.node_l[j], P.node_r[j], P.node_set[j], (uint32_t)M.op[at], M.cost[at], M.card[at]};
    }
    return true;
}

}  // namespace
}  // namespace mpdp
