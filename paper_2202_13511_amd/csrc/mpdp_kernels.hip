// gfx950 kernels of the MPDP level loop (Section 5, Alg. 5):
//   k_init          memo init + base-relation fill
//   k_filter        unrank the k-subsets and keep the connected ones
//   k_eval_tree     Alg. 2 (tree join graphs): one thread per connected set
//   k_eval_general  Alg. 3 (block-based enumeration): one wave64 per set
//   k_extract       rebuild the plan tree from the memo
//
// Everything is integer bitmap work plus a few IEEE binary64 operations per
// join pair; nothing here is a dense contraction, so no MFMA.  Compiled with
// -ffp-contract=off so every cost expression rounds exactly as written.
#include <hip/hip_runtime.h>

#include "mpdp_internal.h"

namespace mpdp {
namespace {

constexpr int kBlock = 256;         // threads per workgroup (4 waves of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kFilterChunk = 8;     // consecutive ranks per lane in the filter
constexpr int kEvalChunk = 16;      // block-local candidates per lane chunk
constexpr uint32_t kMaxGrid = 8192; // workgroups per launch (grid-stride beyond)

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
    uint32_t c = lowbit(x), r = x + c;
    return (((r ^ x) >> 2) / c) | r;
}

// Spread the low bits of j over the set bits of mask (parallel bit deposit).
__device__ __forceinline__ uint32_t deposit(uint32_t j, uint32_t mask) {
    uint32_t r = 0;
    for (uint32_t m = mask; j && m; m &= m - 1, j >>= 1)
        if (j & 1u) r |= lowbit(m);
    return r;
}

// ---------------------------------------------------------------- LDS copy

struct LdsGraph {
    uint32_t nb[4][256];
    uint32_t adj[kMaxRel];
    uint32_t pbit[kMaxRel];
    uint32_t desc[kMaxRel];
    double card[kMaxRel];
    double sel[kMaxRel * kMaxRel];
};

__device__ void stage_graph(const DevGraph *g, LdsGraph &L) {
    const uint32_t *src = &g->nbr_byte[0][0];
    uint32_t *dst = &L.nb[0][0];
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) dst[i] = src[i];
    for (int i = threadIdx.x; i < kMaxRel * kMaxRel; i += blockDim.x) L.sel[i] = g->sel[i];
    if (threadIdx.x < kMaxRel) {
        L.adj[threadIdx.x] = g->adj[threadIdx.x];
        L.pbit[threadIdx.x] = g->tree_parent_bit[threadIdx.x];
        L.desc[threadIdx.x] = g->tree_desc[threadIdx.x];
        L.card[threadIdx.x] = g->card[threadIdx.x];
    }
    __syncthreads();
}

// ---------------------------------------------------------------- cost

// card(S): product over S ascending of card[v] and of the selectivities of
// the edges from v down to smaller members of S; clamped below at 1.
__device__ __forceinline__ double card_of(const LdsGraph &L, uint32_t S) {
    double c = 1.0;
    for (uint32_t T = S; T; T &= T - 1) {
        const int v = ctz32(T);
        c = c * L.card[v];
        for (uint32_t U = L.adj[v] & S & ((1u << v) - 1u); U; U &= U - 1)
            c = c * L.sel[ctz32(U) * kMaxRel + v];
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

// Cost both orientations of the csg-cmp pair (A, B) of S and keep the best.
template <int CM>
__device__ __forceinline__ void eval_pair(const MemoPtrs &M, uint32_t A, uint32_t B, double cardS,
                                          Key &best) {
    const double cA = M.cost[A], cB = M.cost[B];
    const double base = cA + cB;
    if (CM == MPDP_COST_COUT) {
        // symmetric: both orientations cost the same, the smaller left wins
        offer(best, base + cardS, A < B ? A : B, MPDP_OP_JOIN);
    } else {
        const double kA = M.card[A], kB = M.card[B];
        const double out = 0.01 * cardS;
        const double hjA = ((base + 0.0125 * kB) + 0.0025 * kA) + out;  // A outer, B hashed
        const double nlA = (base + (0.0025 * kA) * kB) + out;
        const double hjB = ((base + 0.0125 * kA) + 0.0025 * kB) + out;  // B outer, A hashed
        const double nlB = (base + (0.0025 * kB) * kA) + out;
        if (hjA <= nlA) offer(best, hjA, A, MPDP_OP_HASH); else offer(best, nlA, A, MPDP_OP_NESTLOOP);
        if (hjB <= nlB) offer(best, hjB, B, MPDP_OP_HASH); else offer(best, nlB, B, MPDP_OP_NESTLOOP);
    }
}

__device__ __forceinline__ void store_best(const MemoPtrs &M, uint32_t S, const Key &b, double cardS) {
    M.cost[S] = __longlong_as_double((long long)b.c);
    M.card[S] = cardS;
    M.left[S] = b.l;
    M.op[S] = (uint8_t)b.op;
}

// ---------------------------------------------------------------- kernels

__global__ void k_init(const DevGraph *g, uint32_t n, MemoPtrs M, Counters *cnt) {
    const uint32_t t = threadIdx.x;
    if (t < n) {
        const uint32_t s = 1u << t;
        M.cost[s] = g->base_cost[t];
        M.card[s] = g->card[t];
        M.left[s] = 0;
        M.op[s] = MPDP_OP_SCAN;
    }
    uint32_t *words = reinterpret_cast<uint32_t *>(cnt);
    for (uint32_t i = t; i < sizeof(Counters) / 4; i += blockDim.x) words[i] = 0;
}

// Unrank + filter (Alg. 5 unrank and filter steps, fused).  Each lane takes
// kFilterChunk consecutive colex ranks: it unranks the first with the
// combinatorial number system and steps to the next k-subsets with the
// same-popcount successor.  Connected sets are compacted with a wave ballot
// and one atomic per wave and step.
__global__ __launch_bounds__(kBlock) void k_filter(const DevGraph *g, uint32_t k, uint64_t ncand,
                                                   uint32_t *list, Counters *cnt) {
    __shared__ uint32_t nb[4][256];
    __shared__ uint32_t binom[33 * 33];
    for (int i = threadIdx.x; i < 1024; i += blockDim.x) (&nb[0][0])[i] = (&g->nbr_byte[0][0])[i];
    for (int i = threadIdx.x; i < 33 * 33; i += blockDim.x) binom[i] = g->binom[i];
    __syncthreads();

    const int n = (int)g->n;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t per_wave = 64ull * kFilterChunk;
    const uint64_t waves = (uint64_t)gridDim.x * kWaves;
    uint32_t *level_count = &cnt->level_count[k];

    for (uint64_t w = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); w * per_wave < ncand; w += waves) {
        const uint64_t r0 = w * per_wave + (uint64_t)lane * kFilterChunk;
        uint32_t S = 0;
        if (r0 < ncand) {  // colex unrank of r0
            uint32_t r = (uint32_t)r0;
            int c = n - 1;
            for (int i = (int)k; i >= 1; --i) {
                while (binom[c * 33 + i] > r) --c;
                r -= binom[c * 33 + i];
                S |= 1u << c;
                --c;
            }
        }
        for (int j = 0; j < kFilterChunk; ++j) {
            const bool valid = r0 + (uint64_t)j < ncand;
            bool keep = false;
            if (valid) keep = grow(nb, lowbit(S), S) == S;
            const unsigned long long mask = __ballot(keep);
            if (mask) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(level_count, (uint32_t)__popcll(mask));
                base = __shfl(base, 0);
                if (keep) {
                    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                    list[base + below] = S;
                }
            }
            if (valid) S = next_subset(S);
        }
    }
}

// Alg. 2 on a tree join graph.  With the tree rooted at relation 0, the pair
// obtained by removing the edge (parent(c), c) of G[S] is
// (desc(c) & S, S minus that), for every c in S whose parent is in S.
template <int CM>
__global__ __launch_bounds__(kBlock) void k_eval_tree(const DevGraph *g, uint32_t k, const uint32_t *list,
                                                      const Counters *cnt, MemoPtrs M) {
    __shared__ LdsGraph L;
    stage_graph(g, L);
    const uint32_t count = cnt->level_count[k];
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
        const uint32_t S = list[i];
        const double cardS = card_of(L, S);
        Key best = worst_key();
        for (uint32_t T = S; T; T &= T - 1) {
            const int c = ctz32(T);
            if (!(S & L.pbit[c])) continue;  // c is the root of G[S]
            const uint32_t A = L.desc[c] & S;
            eval_pair<CM>(M, A, S ^ A, cardS, best);
        }
        store_best(M, S, best, cardS);
    }
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

// Alg. 3: one wave64 per connected set S.
//  1. cut vertices of G[S]: lane v checks whether G[S - v] is connected;
//  2. blocks: split S at a cut vertex into pieces {x} + component, recurse
//     until a piece has no cut vertex of its own (piece-local cut vertices
//     are the cut vertices of S inside the piece, minus its attachment);
//  3. lanes share the block-local candidates lb (lb holds the block's lowest
//     relation, lb != block, so each unordered pair is visited once and both
//     orientations are costed); a candidate is a pair when G[lb] and G[rb]
//     are connected; then S_left = grow(lb, S - rb), S_right = S - S_left;
//  4. wave min-reduce of the plan key, lane 0 writes the memo.
template <int CM>
__global__ __launch_bounds__(kBlock) void k_eval_general(const DevGraph *g, uint32_t k, const uint32_t *list,
                                                         Counters *cnt, MemoPtrs M) {
    __shared__ LdsGraph L;
    __shared__ WaveScratch WS[kWaves];
    stage_graph(g, L);
    const int lane = threadIdx.x & 63;
    WaveScratch &W = WS[threadIdx.x >> 6];
    const uint32_t count = cnt->level_count[k];
    unsigned long long my_ccp = 0, my_eval = 0;

    for (uint32_t idx = blockIdx.x * kWaves + (threadIdx.x >> 6); idx < count; idx += gridDim.x * kWaves) {
        const uint32_t S = list[idx];

        // 1. cut vertices
        bool cut = false;
        if (lane < 32 && ((S >> lane) & 1u)) {
            const uint32_t R = S & ~(1u << lane);
            cut = grow(L.nb, lowbit(R), R) != R;
        }
        const uint32_t A = (uint32_t)__ballot(cut);

        // 2. blocks (uniform control flow; the stack lives one entry per lane)
        // A piece is a union of blocks of S; its attachment set holds the
        // split vertices it still contains, which are not cut vertices of
        // the piece.  Every other cut vertex of S inside the piece is.
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

        // 3. per-block candidate counts (lane i owns block i)
        uint32_t half = 0, chunks = 0, complete = 0;
        unsigned long long evalb = 0;
        if (lane < nblk) {
            const int bs = popc32(myblk);
            half = (1u << (bs - 1)) - 1u;
            chunks = (half + kEvalChunk - 1) / kEvalChunk;
            evalb = (1ull << bs) - 2ull;
            uint32_t deg = 0;
            for (uint32_t T = myblk; T; T &= T - 1) deg += popc32(L.adj[ctz32(T)] & myblk);
            complete = deg == (uint32_t)(bs * (bs - 1));
        }
        uint32_t acc = 0, mypre = 0;
        for (int i = 0; i < nblk; ++i) {
            const uint32_t c = rdlane(chunks, i);
            if (lane == i) mypre = acc;
            acc += c;
            my_eval += (lane == 0) ? (1ull << popc32(rdlane(myblk, i))) - 2ull : 0ull;
        }
        (void)evalb;
        const uint32_t total_chunks = acc;
        if (lane < nblk) { W.blk[lane] = myblk; W.full[lane] = complete; W.cpre[lane] = mypre; }
        if (lane == 0) W.cpre[nblk] = total_chunks;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const double cardS = card_of(L, S);
        Key best = worst_key();
        for (uint32_t ch = lane; ch < total_chunks; ch += 64) {
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
                ++my_ccp;
                const uint32_t Sl = (lb & A) ? grow(L.nb, lb, S & ~rb) : lb;
                eval_pair<CM>(M, Sl, S ^ Sl, cardS, best);
            }
        }
        best = wave_min(best);
        if (lane == 0) store_best(M, S, best, cardS);
        __builtin_amdgcn_wave_barrier();
    }

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

// Rebuild the plan (Section 5: fetched recursively through left/right) in
// post-order on one thread; n - 1 memo reads.
__global__ void k_extract(const DevGraph *g, uint32_t n, MemoPtrs M, mpdp_plan_node *plan, double *root_cost,
                          Counters *cnt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (uint32_t v = 0; v < n; ++v) {
        const uint32_t s = 1u << v;
        plan[v] = mpdp_plan_node{-1, -1, s, MPDP_OP_SCAN, M.cost[s], M.card[s]};
    }
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    *root_cost = M.cost[full];
    if (n == 1) return;
    struct Frame { uint32_t S; int stage; int li; };
    Frame st[33];
    int sp = 0, next = (int)n, ret = -1, guard = 0;
    st[sp++] = Frame{full, 0, -1};
    while (sp > 0 && ++guard < 4 * 64) {
        Frame &f = st[sp - 1];
        const uint32_t Lft = M.left[f.S];
        if (Lft == 0 || (Lft & ~f.S) != 0 || Lft == f.S) { cnt->extract_error = 1; return; }
        const uint32_t Rgt = f.S & ~Lft;
        if (f.stage == 0) {
            f.stage = 1;
            if ((Lft & (Lft - 1)) == 0) ret = ctz32(Lft);
            else { if (sp >= 33) { cnt->extract_error = 2; return; } st[sp++] = Frame{Lft, 0, -1}; continue; }
        }
        if (f.stage == 1) {
            f.li = ret;
            f.stage = 2;
            if ((Rgt & (Rgt - 1)) == 0) ret = ctz32(Rgt);
            else { if (sp >= 33) { cnt->extract_error = 2; return; } st[sp++] = Frame{Rgt, 0, -1}; continue; }
        }
        plan[next] = mpdp_plan_node{f.li, ret, f.S, (uint32_t)M.op[f.S], M.cost[f.S], M.card[f.S]};
        ret = next++;
        --sp;
    }
    if (sp != 0 || next != (int)(2 * n - 1)) cnt->extract_error = 3;
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

hipError_t launch_eval_tree(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand,
                            const uint32_t *list, const Counters *cnt, MemoPtrs memo, hipStream_t s) {
    const uint32_t grid = grid_for(ncand, kBlock);
    if (cost_model == MPDP_COST_COUT)
        hipLaunchKernelGGL(k_eval_tree<MPDP_COST_COUT>, dim3(grid), dim3(kBlock), 0, s, g, k, list, cnt, memo);
    else
        hipLaunchKernelGGL(k_eval_tree<MPDP_COST_PGLIKE>, dim3(grid), dim3(kBlock), 0, s, g, k, list, cnt, memo);
    return hipGetLastError();
}

hipError_t launch_eval_general(const DevGraph *g, int cost_model, uint32_t k, uint64_t ncand,
                               const uint32_t *list, Counters *cnt, MemoPtrs memo, hipStream_t s) {
    const uint32_t grid = grid_for(ncand, kWaves);
    if (cost_model == MPDP_COST_COUT)
        hipLaunchKernelGGL(k_eval_general<MPDP_COST_COUT>, dim3(grid), dim3(kBlock), 0, s, g, k, list, cnt, memo);
    else
        hipLaunchKernelGGL(k_eval_general<MPDP_COST_PGLIKE>, dim3(grid), dim3(kBlock), 0, s, g, k, list, cnt,
                           memo);
    return hipGetLastError();
}

hipError_t launch_extract(const DevGraph *g, uint32_t n, MemoPtrs memo, mpdp_plan_node *plan,
                          double *root_cost, Counters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_extract, dim3(1), dim3(64), 0, s, g, n, memo, plan, root_cost, cnt);
    return hipGetLastError();
}

}  // namespace mpdp
