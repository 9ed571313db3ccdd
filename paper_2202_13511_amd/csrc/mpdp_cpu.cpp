// MPDP on the host's cores: the all-cores CPU baseline the GPU path is
// measured against (Section 3.3: work items handed out through an atomic
// counter).  Same level-by-level DP, enumeration (Alg. 2 on tree joins,
// Alg. 3 otherwise), card(S), cost formulas and plan key as the GPU path
// (include/mpdp.h), so its memo is bit-identical; the memo is a dense
// array indexed by the relation bitmap.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "mpdp.h"

namespace {

constexpr uint32_t kCpuMaxRel = 28;
constexpr uint64_t kChunk = 4096;  // candidates per work item

struct CpuGraph {
    uint32_t n, cm;
    uint32_t adj[32];
    double card[32], bcost[32];
    double sel[32][32];
};

inline uint32_t low(uint32_t x) { return x & (0u - x); }
inline int ctz(uint32_t x) { return __builtin_ctz(x); }
inline int popc(uint32_t x) { return __builtin_popcount(x); }

uint32_t grow(const CpuGraph &g, uint32_t src, uint32_t R) {
    uint32_t seen = src, fr = src;
    while (fr) {
        uint32_t nb = 0;
        for (uint32_t t = fr; t; t &= t - 1) nb |= g.adj[ctz(t)];
        fr = nb & R & ~seen;
        seen |= fr;
    }
    return seen;
}

double card_of(const CpuGraph &g, uint32_t S) {
    double c = 1.0;
    for (uint32_t T = S; T; T &= T - 1) {
        const int v = ctz(T);
        c = c * g.card[v];
        for (uint32_t U = g.adj[v] & S & ((1u << v) - 1u); U; U &= U - 1) c = c * g.sel[ctz(U)][v];
    }
    return c < 1.0 ? 1.0 : c;
}

struct Best {
    double cost;
    uint32_t left, op;
    bool have;
};

inline bool less_key(double c, uint32_t l, uint32_t op, const Best &b) {
    if (!b.have) return true;
    if (c != b.cost) return c < b.cost;
    if (l != b.left) return l < b.left;
    return op < b.op;
}

struct Memo {
    std::vector<double> cost, card;
    std::vector<uint32_t> left;
    std::vector<uint8_t> op;
};

// Both orientations of the pair (A, B) of S.
inline void consider(const CpuGraph &g, const Memo &M, uint32_t A, uint32_t B, double cS, Best &b) {
    const double cA = M.cost[A], cB = M.cost[B], base = cA + cB;
    if (g.cm == MPDP_COST_COUT) {
        const double c = base + cS;
        const uint32_t l = A < B ? A : B;
        if (less_key(c, l, MPDP_OP_JOIN, b)) b = Best{c, l, MPDP_OP_JOIN, true};
        return;
    }
    const double kA = M.card[A], kB = M.card[B], out = 0.01 * cS;
    const uint32_t L[2] = {A, B};
    const double kl[2] = {kA, kB}, kr[2] = {kB, kA};
    for (int i = 0; i < 2; ++i) {
        const double hj = ((base + 0.0125 * kr[i]) + 0.0025 * kl[i]) + out;
        const double nl = (base + (0.0025 * kl[i]) * kr[i]) + out;
        const double c = hj <= nl ? hj : nl;
        const uint32_t op = hj <= nl ? MPDP_OP_HASH : MPDP_OP_NESTLOOP;
        if (less_key(c, L[i], op, b)) b = Best{c, L[i], op, true};
    }
}

// Blocks of G[S] (S connected, |S| >= 2): depth-first search from the
// lowest relation with lowpoints; a child v of p whose subtree has no edge
// above p closes a block.
int blocks_of(const CpuGraph &g, uint32_t S, uint32_t *out) {
    int disc[32], lowp[32], parent[32], order = 0, nb = 0;
    uint32_t stackv[32];
    int sp = 0;
    uint32_t estack[64];  // vertices on the block stack
    int esp = 0;
    uint32_t iter[32];
    for (uint32_t T = S; T; T &= T - 1) disc[ctz(T)] = -1;
    const int root = ctz(S);
    disc[root] = lowp[root] = order++;
    parent[root] = -1;
    iter[root] = g.adj[root] & S;
    stackv[sp++] = (uint32_t)root;
    estack[esp++] = (uint32_t)root;
    while (sp > 0) {
        const int v = (int)stackv[sp - 1];
        if (iter[v]) {
            const int u = ctz(iter[v]);
            iter[v] &= iter[v] - 1;
            if (disc[u] < 0) {
                disc[u] = lowp[u] = order++;
                parent[u] = v;
                iter[u] = g.adj[u] & S;
                stackv[sp++] = (uint32_t)u;
                estack[esp++] = (uint32_t)u;
            } else if (u != parent[v]) {
                lowp[v] = std::min(lowp[v], disc[u]);
            }
        } else {
            --sp;
            const int p = parent[v];
            if (p >= 0) {
                lowp[p] = std::min(lowp[p], lowp[v]);
                if (lowp[v] >= disc[p]) {  // p separates v's subtree: pop one block
                    uint32_t blk = 1u << p;
                    while (esp > 0) {
                        const uint32_t w = estack[--esp];
                        blk |= 1u << w;
                        if ((int)w == v) break;
                    }
                    out[nb++] = blk;
                }
            }
        }
    }
    return nb;
}

void eval_set(const CpuGraph &g, Memo &M, uint32_t S, bool tree, uint64_t &evaluated, uint64_t &ccp) {
    const double cS = card_of(g, S);
    Best b{0.0, 0, 0, false};
    if (tree) {  // Alg. 2: one pair per edge (u, v) of G[S]
        for (uint32_t T = S; T; T &= T - 1) {
            const int v = ctz(T);
            for (uint32_t U = g.adj[v] & S & ((1u << v) - 1u); U; U &= U - 1) {
                const uint32_t L = grow(g, low(U), S & ~(1u << v));
                consider(g, M, L, S & ~L, cS, b);
                evaluated += 2;
                ccp += 1;
            }
        }
    } else {  // Alg. 3 over the blocks of G[S]; lb holds the block's lowest relation
        uint32_t blk[32];
        const int nb = blocks_of(g, S, blk);
        for (int i = 0; i < nb; ++i) {
            const uint32_t B = blk[i], lo = low(B), rest = B ^ lo;
            evaluated += (1ull << popc(B)) - 2ull;
            for (uint32_t sub = 0;; sub = (sub - rest) & rest) {
                const uint32_t lb = lo | sub, rb = B ^ lb;
                if (rb != 0 && grow(g, lo, lb) == lb && grow(g, low(rb), rb) == rb) {
                    const uint32_t L = grow(g, lb, S & ~rb);
                    consider(g, M, L, S & ~L, cS, b);
                    ccp += 1;
                }
                if (sub == rest) break;
            }
        }
    }
    M.cost[S] = b.cost;
    M.card[S] = cS;
    M.left[S] = b.left;
    M.op[S] = (uint8_t)b.op;
}

uint64_t binom(uint32_t a, uint32_t b) {
    if (b > a) return 0;
    uint64_t r = 1;
    for (uint32_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
}

// k-subset of rank r in colex order
uint32_t unrank(uint32_t n, uint32_t k, uint64_t r) {
    uint32_t S = 0;
    for (uint32_t i = k; i >= 1; --i) {
        uint32_t c = i - 1;
        while (c + 1 < n && binom(c + 1, i) <= r) ++c;
        r -= binom(c, i);
        S |= 1u << c;
        n = c;
    }
    return S;
}

uint32_t next_same_popcount(uint32_t x) {
    const uint32_t l = low(x), r = x + l;
    return (((r ^ x) >> 2) >> ctz(x)) | r;
}

}  // namespace

extern "C" mpdp_status mpdp_optimize_cpu(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *cardinalities,
                                         const double *selectivities, mpdp_cost_model cost_model, uint32_t threads,
                                         mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!plan_out || !cost_out || !cardinalities || (m > 0 && (!edges || !selectivities))) return MPDP_EINVAL;
    if (n == 0) return MPDP_EINVAL;
    if (n > kCpuMaxRel) return MPDP_ETOOLARGE;
    if (cost_model != MPDP_COST_COUT && cost_model != MPDP_COST_PGLIKE) return MPDP_EINVAL;
    if (m > n * (n - 1) / 2) return MPDP_EINVAL;
    CpuGraph g;
    std::memset(&g, 0, sizeof(g));
    g.n = n;
    g.cm = cost_model;
    for (uint32_t v = 0; v < n; ++v) {
        if (!std::isfinite(cardinalities[v]) || !(cardinalities[v] >= 1.0)) return MPDP_EINVAL;
        g.card[v] = cardinalities[v];
        g.bcost[v] = cost_model == MPDP_COST_PGLIKE ? 0.01 * cardinalities[v] : 0.0;
    }
    for (uint32_t i = 0; i < m; ++i) {
        const uint32_t u = edges[i].u, v = edges[i].v;
        const double s = selectivities[i];
        if (u >= n || v >= n || u == v || (g.adj[u] >> v) & 1u) return MPDP_EINVAL;
        if (!std::isfinite(s) || !(s > 0.0) || !(s <= 1.0)) return MPDP_EINVAL;
        g.adj[u] |= 1u << v;
        g.adj[v] |= 1u << u;
        g.sel[u][v] = g.sel[v][u] = s;
    }
    const uint32_t full = (n == 32) ? ~0u : ((1u << n) - 1u);
    if (grow(g, 1u, full) != full) return MPDP_ENOTCONNECTED;
    const bool tree = m == n - 1;
    if (threads == 0) threads = std::max(1u, std::thread::hardware_concurrency());

    Memo M;
    try {
        const size_t N = (size_t)1 << n;
        M.cost.assign(N, 0.0);
        M.card.assign(N, 0.0);
        M.left.assign(N, 0);
        M.op.assign(N, 0);
    } catch (...) {
        return MPDP_ENOMEM;
    }
    for (uint32_t v = 0; v < n; ++v) {
        M.cost[1u << v] = g.bcost[v];
        M.card[1u << v] = g.card[v];
        M.op[1u << v] = MPDP_OP_SCAN;
    }
    std::atomic<uint64_t> evaluated{0}, ccp{0}, conn{0};
    for (uint32_t k = 2; k <= n; ++k) {
        const uint64_t total = binom(n, k);
        std::atomic<uint64_t> next{0};
        auto work = [&]() {
            uint64_t e = 0, c = 0, s = 0;
            for (;;) {
                const uint64_t r0 = next.fetch_add(kChunk);
                if (r0 >= total) break;
                const uint64_t r1 = std::min(total, r0 + kChunk);
                uint32_t S = unrank(n, k, r0);
                for (uint64_t r = r0; r < r1; ++r, S = next_same_popcount(S)) {
                    if (grow(g, low(S), S) != S) continue;
                    ++s;
                    eval_set(g, M, S, tree, e, c);
                }
            }
            evaluated += e;
            ccp += c;
            conn += s;
        };
        std::vector<std::thread> pool;
        for (uint32_t t = 1; t < threads; ++t) pool.emplace_back(work);
        work();
        for (auto &th : pool) th.join();
    }
    // plan: leaves, then joins in post-order from the full set
    for (uint32_t v = 0; v < n; ++v)
        plan_out[v] = mpdp_plan_node{-1, -1, 1u << v, MPDP_OP_SCAN, M.cost[1u << v], M.card[1u << v]};
    int next = (int)n;
    std::vector<std::pair<uint32_t, int>> st{{full, 0}};
    std::vector<int> idx;
    while (!st.empty()) {
        auto &[S, stage] = st.back();
        if ((S & (S - 1)) == 0) {
            idx.push_back(ctz(S));
            st.pop_back();
            continue;
        }
        const uint32_t L = M.left[S];
        if (stage == 0) { stage = 1; st.push_back({L, 0}); continue; }
        if (stage == 1) { stage = 2; st.push_back({S & ~L, 0}); continue; }
        const int r = idx.back(); idx.pop_back();
        const int l = idx.back(); idx.pop_back();
        plan_out[next] = mpdp_plan_node{l, r, S, M.op[S], M.cost[S], M.card[S]};
        idx.push_back(next++);
        st.pop_back();
    }
    *cost_out = M.cost[full];
    if (stats_out) {
        mpdp_stats st2{};
        uint64_t cand = 0;
        for (uint32_t k = 2; k <= n; ++k) cand += binom(n, k);
        st2.candidates = cand;
        st2.connected_sets = conn.load();
        st2.evaluated_pairs = evaluated.load();
        st2.ccp_pairs = ccp.load();
        st2.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st2.levels = n - 1;
        st2.eval_launches = threads;
        *stats_out = st2;
    }
    return MPDP_OK;
}
