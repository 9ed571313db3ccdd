// Batched optimization of many small queries in one persistent launch.
//
// Each workgroup pulls the next query from an atomic counter and runs the
// whole level loop of Alg. 5 for it, with workgroup barriers between levels
// instead of kernel launches: it builds the query's LDS image from the raw
// edges, cardinalities and selectivities, fills the base relations, runs
// levels 2..n (Alg. 2 for tree joins, Alg. 3 otherwise: filter, one wave per
// light set, the whole workgroup per heavy set), rebuilds the plan and
// records the device wall clock at the query's start and end.  Memo and
// scratch live in a per-workgroup slot that is reused from query to query,
// so the workspace does not grow with the batch.  A large cyclic query is
// taken by a team of workgroups (consecutive queue entries): they split the
// candidates and sets of every level and meet at device-wide barriers, in
// the slot of the team's first member.  Entries are taken in queue order,
// so a member waiting at a barrier waits only for workgroups that have
// already taken their entries, or for ones that will take them next.
#include <hip/hip_runtime.h>

#include "mpdp_device.h"
#include "mpdp_internal.h"

namespace mpdp {
namespace {

constexpr int kBatchBlock = 512;
constexpr int kBW = kBatchBlock / 64;
// members per gather batch of a tree set: three keeps the kernel (every
// path of a query inlined, 128 registers per lane) from spilling far more
constexpr int kBatchPairBatch = 3;
// (for the same reason Alg. 3's candidate chunks take the plain subset walk
// here, without the per-chunk neighbourhood tables)
constexpr unsigned long long kTeamWaitTicks = 200000000ull;  // 2 s of the 100 MHz device clock

// The workgroups of a team meet here for the `phase`-th time.  Every wave
// first waits until its own stores (memo, lists) have reached the L2; then
// one thread per workgroup writes the L2 back (agent-scope release) and
// arrives, and after the wait drops the lines other members may have
// written from this CU's and this XCD's caches (agent-scope acquire), once
// for all its waves.  The wait is bounded by the device clock: past
// kTeamWaitTicks the team is marked failed, and every later wait of that
// team returns at once.  Returns false once the team has failed; its
// members then leave the query (its lists may be incomplete), and the
// query reports an error.
__device__ bool team_barrier(TeamRec *R, uint32_t team, uint32_t &phase, uint32_t &s_ok) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&R->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = team * (phase + 1u);
        const unsigned long long start = wall_clock64();
        while (__hip_atomic_load(&R->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target &&
               __hip_atomic_load(&R->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            __builtin_amdgcn_s_sleep(2);
            if ((unsigned long long)wall_clock64() - start > kTeamWaitTicks) {
                __hip_atomic_store(&R->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        s_ok = __hip_atomic_load(&R->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ++phase;
    __syncthreads();
    return s_ok != 0u;
}

__device__ __forceinline__ uint32_t load_shared_count(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Build the LDS image of one query inside the workgroup (everything except
// the binomials, which are staged once per workgroup).
__device__ void build_image(LdsGraph &L, const BatchQueryDev &Q, const uint32_t *edges, const double *cards,
                            const double *sels, const double *bcosts) {
    const uint32_t t = threadIdx.x, n = Q.n, m = Q.m;
    const uint32_t *E = edges + 2ull * Q.edge_off;
    const double *C = cards + Q.card_off;
    const double *SL = sels + Q.edge_off;
    if (t < kMaxRel) {
        L.adj[t] = 0;
        L.pd[t][0] = 0;
        L.lo[t][0] = 0;
        L.lo[t][1] = 0;
        L.csel[t][0] = t < n ? C[t] : 1.0;
        L.csel[t][1] = 1.0;
        L.pd[t][1] = 1u << t;
        L.card[t] = t < n ? C[t] : 1.0;
        if (t >= n) L.bcost[t] = 0.0;
        else if (bcosts) L.bcost[t] = bcosts[Q.card_off + t];  // planned intermediate results
        else L.bcost[t] = Q.cost_model == MPDP_COST_PGLIKE ? 0.01 * C[t] : 0.0;
    }
    __syncthreads();
    for (uint32_t e = t; e < m; e += blockDim.x) {
        const uint32_t u = E[2 * e], v = E[2 * e + 1];
        atomicOr(&L.adj[u], 1u << v);
        atomicOr(&L.adj[v], 1u << u);
    }
    __syncthreads();
    if (t < n) {  // selectivities of edges (u, v), u < v, grouped by v, u ascending
        const uint32_t lower = L.adj[t] & ((1u << t) - 1u);
        uint32_t start = 0;
        for (uint32_t w = 0; w < t; ++w) start += (uint32_t)popc32(L.adj[w] & ((1u << w) - 1u));
        L.selrow[t] = start;
        for (uint32_t e = 0; e < m; ++e) {
            const uint32_t a = E[2 * e], b = E[2 * e + 1];
            const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
            if (hi == t) L.sel[start + (uint32_t)popc32(lower & ((1u << lo) - 1u))] = SL[e];
        }
        L.lo[t][0] = lower & (0u - lower);
        L.lo[t][1] = lower & ~(lower & (0u - lower));
        L.csel[t][1] = lower ? L.sel[start] : 1.0;  // written by this thread above
    }
    for (uint32_t i = t; i < 4 * 256; i += blockDim.x) {
        const uint32_t byte = i >> 8, x = i & 255u;
        uint32_t u = 0;
        for (uint32_t j = 0; j < 8; ++j)
            if (((x >> j) & 1u) && 8u * byte + j < n) u |= L.adj[8u * byte + j];
        L.nb[byte][x] = u;
    }
    if (t == 0) {
        uint64_t off = 0;
        for (uint32_t k = 0; k < 34; ++k) {
            L.loff[k] = off;
            if (k <= n) off += L.binom[n * 33 + k];
        }
        if (Q.is_tree) {  // rooted at relation 0: parent bits and subtree sets in BFS order
            uint32_t order[kMaxRel], parent[kMaxRel];
            uint32_t head = 0, tail = 0, vis = 1u;
            order[tail++] = 0;
            parent[0] = 0;
            while (head < tail) {
                const uint32_t v = order[head++];
                for (uint32_t T = L.adj[v] & ~vis; T; T &= T - 1) {
                    const uint32_t c = (uint32_t)ctz32(T);
                    parent[c] = v;
                    vis |= 1u << c;
                    order[tail++] = c;
                }
            }
            for (uint32_t i = 1; i < tail; ++i) L.pd[order[i]][0] = 1u << parent[order[i]];
            for (uint32_t i = tail - 1; i > 0; --i) L.pd[parent[order[i]]][1] |= L.pd[order[i]][1];
        }
    }
    __syncthreads();
    if (Q.is_tree) {  // children of a set, one table per bitmap byte
        for (uint32_t i = t; i < 4 * 256; i += blockDim.x) {
            const uint32_t byte = i >> 8, x = i & 255u;
            uint32_t c = 0;
            for (uint32_t v = 1; v < n; ++v)
                if (L.pd[v][0] & (x << (8u * byte))) c |= 1u << v;
            L.ch[byte][x] = c;
        }
        __syncthreads();
    }
}

template <int CM>
__global__ __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_batch(const BatchQueryDev *qs, const uint32_t *edges,
                                                       const double *cards, const double *sels,
                                                       const double *bcosts, const uint32_t *binom_g, char *slots, uint64_t slot_bytes,
                                                       uint32_t maxn, mpdp_plan_node *plans, BatchOut *out,
                                                       TeamRec *teams, BatchCounters *bc) {
    __shared__ __align__(16) LdsGraph L;
    __shared__ uint32_t rings[kBW][kRing];
    __shared__ uint32_t ring_bsums[kBW][kRing];
    __shared__ WaveScratch WS[kBW];
    __shared__ SetBlocks hsb;
    __shared__ Key hkeys[kBW];
    __shared__ PlanScratch P;
    __shared__ uint32_t s_q, s_level, s_ok;
    __shared__ uint32_t s_ntree[24], s_ngen[24], s_nheavy[24];  // per level k: list and heavy-list counts
    __shared__ unsigned long long s_conn, s_ccp, s_eval, s_t0;
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    if (t == 0) atomicMin(&bc->t0, (unsigned long long)wall_clock64());
    // the entry count travels with the uploaded data, so a recorded launch
    // serves any run with the same layout
    const uint32_t nq = bc->entries;
    for (uint32_t i = t; i < 33 * 33; i += blockDim.x) L.binom[i] = binom_g[i];

    // a workgroup's slot: memo (cost, card, left, op over 2^maxn entries), set list, heavy list
    const uint64_t N = 1ull << maxn;
    const uint64_t list_off = (21 * N + 255) & ~255ull;
    // sets of the widest level; read from global memory: the LDS copy of the
    // table is complete only after the first barrier below
    const uint32_t cap = binom_g[maxn * 33 + maxn / 2];

    for (;;) {
        if (t == 0) s_q = atomicAdd(&bc->next, 1u);
        __syncthreads();
        const uint32_t q = s_q;
        if (q >= nq) break;
        const BatchQueryDev Q = qs[q];
        const bool team = Q.team > 1;
        TeamRec *R = team ? teams + Q.team_rec : nullptr;
        uint32_t phase = 0;
        build_image(L, Q, edges, cards, sels, bcosts);
        const uint32_t n = Q.n;
        if (t == 0) {
            s_t0 = (unsigned long long)wall_clock64();
            s_conn = 0;
            s_ccp = 0;
            s_eval = 0;
        }
        // a team works in its first member's slot, published through the team record
        uint32_t slot_id = blockIdx.x;
        if (team && Q.member == 0 && t == 0) __hip_atomic_store(&R->slot, slot_id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        char *slot = slots + (uint64_t)slot_id * slot_bytes;
        MemoPtrs M{reinterpret_cast<double *>(slot), reinterpret_cast<double *>(slot + 8 * N),
                   reinterpret_cast<uint32_t *>(slot + 16 * N), reinterpret_cast<uint8_t *>(slot + 20 * N)};
        if (t < 24) {
            s_ntree[t] = 0;
            s_ngen[t] = 0;
            s_nheavy[t] = 0;
        }
        if (t < n && Q.member == 0) {
            const uint64_t at = L.loff[1] + t;
            M.cost[at] = L.bcost[t];
            M.card[at] = L.card[t];
            M.left[at] = 0;
            M.op[at] = MPDP_OP_SCAN;
        }
        bool failed = false;
        if (team) {
            failed = !team_barrier(R, Q.team, phase, s_ok);
            slot_id = load_shared_count(&R->slot);
            slot = slots + (uint64_t)slot_id * slot_bytes;
            M = MemoPtrs{reinterpret_cast<double *>(slot), reinterpret_cast<double *>(slot + 8 * N),
                         reinterpret_cast<uint32_t *>(slot + 16 * N), reinterpret_cast<uint8_t *>(slot + 20 * N)};
        } else {
            __syncthreads();
        }
        // two set lists of cap entries (level k uses list k mod 2, so the
        // filter of level k + 1 can run with level k's evaluation), then the
        // heavy list
        uint32_t *lists = reinterpret_cast<uint32_t *>(slot + list_off);
        uint32_t *hv = lists + 2 * cap;
        // this workgroup's waves among the team's (w0, w0 + wstride, ...)
        const uint32_t w0 = Q.member * kBW + wave, wstride = Q.team * kBW;
        auto filter_level = [&](uint32_t kk) {  // connected sets of level kk into their list
            filter_wave(L, (int)n, kk, L.binom[n * 33 + kk], w0, wstride, lists + (kk & 1u) * cap, cap,
                        team ? &R->ntree[kk] : &s_ntree[kk], team ? &R->ngen[kk] : &s_ngen[kk], lane);
        };
        if (!Q.is_tree && n >= 2 && !failed) {
            filter_level(2);
            if (team) failed = !team_barrier(R, Q.team, phase, s_ok);
            else __syncthreads();
        }
        unsigned long long my_ccp = 0, my_eval = 0;
        for (uint32_t k = 2; k <= n && !failed; ++k) {
            const uint64_t ncand = L.binom[n * 33 + k];
            if (Q.is_tree) {
                if (t == 0) s_level = 0;
                __syncthreads();
                uint32_t found;
                switch (Q.sched & kSchedChunkMask) {  // consecutive ranks per lane
                    case 0:
                        found = level_tree_wave<CM, 1, true, kRing, 1, kBatchPairBatch>(L, M, (int)n, k, ncand, wave, kBW, (ncand + 63) / 64,
                                                       rings[wave], ring_bsums[wave], lane);
                        break;
                    case 1:
                        found = level_tree_wave<CM, 2, true, kRing, 1, kBatchPairBatch>(L, M, (int)n, k, ncand, wave, kBW, (ncand + 127) / 128,
                                                       rings[wave], ring_bsums[wave], lane);
                        break;
                    default:
                        found = level_tree_wave<CM, 4, true, kRing, 1, kBatchPairBatch>(L, M, (int)n, k, ncand, wave, kBW, (ncand + 255) / 256,
                                                       rings[wave], ring_bsums[wave], lane);
                        break;
                }
                if (lane == 0 && found) atomicAdd(&s_level, found);
                __syncthreads();
                if (t == 0) {
                    s_conn += s_level;
                    s_ccp += (unsigned long long)(k - 1) * s_level;
                    s_eval += 2ull * (k - 1) * s_level;
                }
                __syncthreads();
                continue;
            }
            // level k's list was filtered during level k - 1 (or before the loop)
            uint32_t *nhp = team ? &R->nheavy[k] : &s_nheavy[k];
            const uint32_t ntree = team ? load_shared_count(&R->ntree[k]) : s_ntree[k];
            const uint32_t ngen = team ? load_shared_count(&R->ngen[k]) : s_ngen[k];
            const uint32_t count = ntree + ngen;
            // light work: tree-inducing sets one per lane, other sets one per wave
            light_sets<CM, false>(L, M, lists + (k & 1u) * cap, cap, ntree, ngen, w0, wstride, WS[wave], hv, nhp, lane,
                           my_ccp, my_eval, false, (Q.sched >> kSchedHeavyShift) & 0xffffu);
            if (k < n) filter_level(k + 1);
            if (team) {
                if (!team_barrier(R, Q.team, phase, s_ok)) { failed = true; break; }
            } else {
                __syncthreads();
            }
            // heavy sets: a whole workgroup each (a team deals them out)
            const uint32_t hcount = team ? load_shared_count(nhp) : s_nheavy[k];
            for (uint32_t h = Q.member; h < hcount; h += Q.team) {
                const uint32_t S = hv[h];
                if (wave == 0) {
                    const SetBlocks sb = analyze_set(L, S, WS[0], lane, blockDim.x);
                    if (lane == 0) { hsb = sb; my_eval += sb.evaluated; }
                }
                __syncthreads();
                const SetBlocks sb = hsb;
                const double cardS = card_of_wave(L, S, threadIdx.x & 63u);
                Key best = worst_key();
                eval_chunks<CM, false>(L, M, WS[0], S, sb, t, blockDim.x, cardS, best, my_ccp);
                best = wave_min(best);
                if (lane == 0) hkeys[wave] = best;
                __syncthreads();
                if (t == 0) {
                    Key b = hkeys[0];
                    for (int i = 1; i < kBW; ++i)
                        if (key_less(hkeys[i], b)) b = hkeys[i];
                    store_best(M, memo_index(L, S), b, cardS);
                }
                __syncthreads();
            }
            if (t == 0) s_conn += count;
            // the level's memo is complete before the next level reads it
            if (team) failed = !team_barrier(R, Q.team, phase, s_ok);
            else __syncthreads();
        }
        // counters of the block-based path
        for (int off = 32; off >= 1; off >>= 1) {
            my_ccp += (unsigned long long)__shfl_xor((long long)my_ccp, off);
            my_eval += (unsigned long long)__shfl_xor((long long)my_eval, off);
        }
        if (lane == 0 && (my_ccp || my_eval)) {
            atomicAdd(&s_ccp, my_ccp);
            atomicAdd(&s_eval, my_eval);
        }
        __syncthreads();
        if (team) {  // the team's counters meet in its record; the first member finishes the query
            if (t == 0) {
                __hip_atomic_fetch_add(&R->ccp, s_ccp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&R->evaluated, s_eval, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (!failed) failed = !team_barrier(R, Q.team, phase, s_ok);
            if (Q.member != 0) continue;
            if (t == 0) {
                s_ccp = __hip_atomic_load(&R->ccp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_eval = __hip_atomic_load(&R->evaluated, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
        }
        double root = 0.0;
        const bool ok = !failed && extract_plan(L.binom, L.loff, M, n, plans + Q.plan_off, &root, P, t, blockDim.x);
        __syncthreads();
        if (t == 0) {
            BatchOut o;
            o.cost = root;
            o.t_start = s_t0;
            o.t_end = (unsigned long long)wall_clock64();
            o.connected = s_conn;
            o.ccp = s_ccp;
            o.evaluated = s_eval;
            o.error = ok ? 0u : 1u;
            o.pad = 0;
            out[Q.out] = o;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_batch(int cost_model, uint32_t workgroups, const BatchQueryDev *qs,
                        const uint32_t *edges, const double *cards, const double *sels, const double *bcosts,
                        const uint32_t *binom,
                        char *slots, uint64_t slot_bytes, uint32_t maxn, mpdp_plan_node *plans, BatchOut *out,
                        TeamRec *teams, BatchCounters *bc, hipStream_t s) {
    if (cost_model == MPDP_COST_COUT)
        hipLaunchKernelGGL(k_batch<MPDP_COST_COUT>, dim3(workgroups), dim3(kBatchBlock), 0, s, qs, edges, cards,
                           sels, bcosts, binom, slots, slot_bytes, maxn, plans, out, teams, bc);
    else
        hipLaunchKernelGGL(k_batch<MPDP_COST_PGLIKE>, dim3(workgroups), dim3(kBatchBlock), 0, s, qs, edges,
                           cards, sels, bcosts, binom, slots, slot_bytes, maxn, plans, out, teams, bc);
    return hipGetLastError();
}

}  // namespace mpdp
