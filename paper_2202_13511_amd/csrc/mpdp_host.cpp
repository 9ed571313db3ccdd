// Host side of the C-ABI in include/mpdp.h: input validation, the query
// information upload, the level loop of Alg. 5 (unrank+filter, evaluate per
// level, all enqueued on one stream with no host round trip between levels)
// and the plan readback.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <vector>

#include "mpdp.h"
#include "mpdp_host_internal.h"
#include "mpdp_internal.h"

namespace {

using mpdp::Counters;
using mpdp::DevGraph;
using mpdp::MemoPtrs;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

uint64_t binom64(uint32_t a, uint32_t b) {
    if (b > a) return 0;
    uint64_t r = 1;
    for (uint32_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
}

struct Layout {
    size_t cost, card, left, op, list, heavy, parts, graph, counters, plan, root, total;
};

Layout make_layout(uint32_t n) {
    const size_t N = size_t(1) << n;
    Layout L{};
    size_t o = 0;
    L.cost = o;     o = align_up(o + 8 * N);
    L.card = o;     o = align_up(o + 8 * N);
    L.left = o;     o = align_up(o + 4 * N);
    L.op = o;       o = align_up(o + N);
    L.list = o;     o = align_up(o + 4 * binom64(n, n / 2));
    L.heavy = o;    o = align_up(o + 4 * binom64(n, n / 2));
    L.parts = o;    o = align_up(o + sizeof(mpdp::HeavyPart) * mpdp::kHeavyGrid);
    L.graph = o;    o = align_up(o + sizeof(DevGraph));
    L.counters = o; o = align_up(o + sizeof(Counters));
    L.plan = o;     o = align_up(o + sizeof(mpdp_plan_node) * 64);
    L.root = o;     o = align_up(o + sizeof(double));
    L.total = o;
    return L;
}

struct Query {
    uint32_t n, m;
    int cost_model;
    bool is_tree;
    DevGraph g;
    double sel_full[32 * 32];  // host only: sel[u * 32 + v], symmetric, 0 without an edge
};

// C(a, b) for a, b <= 32 at [a * 33 + b], computed once (static storage,
// no heap).
struct BinomTable {
    uint32_t v[33 * 33];
};
const uint32_t *binom_table() {
    static const BinomTable t = [] {
        BinomTable b{};
        for (uint32_t a = 0; a <= 32; ++a)
            for (uint32_t c = 0; c <= 32; ++c) b.v[a * 33 + c] = (uint32_t)binom64(a, c);
        return b;
    }();
    return t.v;
}

// Validation runs entirely on the host, before any HIP call.  base_costs
// (may be null) gives each relation the cost of an already planned
// intermediate result instead of its scan.
mpdp_status validate(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *card, const double *sel,
                     mpdp_cost_model cm, const double *base_costs, Query &q) {
    if (n == 0) return MPDP_EINVAL;
    if (n > 32) return MPDP_ETOOLARGE;
    if (cm != MPDP_COST_COUT && cm != MPDP_COST_PGLIKE) return MPDP_EINVAL;
    if (!card || (m > 0 && (!edges || !sel))) return MPDP_EINVAL;
    if (m > n * (n - 1) / 2) return MPDP_EINVAL;
    std::memset(&q, 0, sizeof(q));
    q.n = n;
    q.m = m;
    q.cost_model = cm;
    DevGraph &g = q.g;
    mpdp::LdsImage &L = g.lds;
    g.n = n;
    g.m = m;
    g.cost_model = (uint32_t)cm;
    for (uint32_t v = 0; v < n; ++v) {
        if (!std::isfinite(card[v]) || !(card[v] >= 1.0)) return MPDP_EINVAL;
        L.card[v] = card[v];
        if (base_costs) {
            if (!std::isfinite(base_costs[v]) || !(base_costs[v] >= 0.0)) return MPDP_EINVAL;
            L.bcost[v] = base_costs[v];
        } else {
            L.bcost[v] = (cm == MPDP_COST_PGLIKE) ? 0.01 * card[v] : 0.0;
        }
    }
    for (uint32_t i = 0; i < m; ++i) {
        const uint32_t u = edges[i].u, v = edges[i].v;
        if (u >= n || v >= n || u == v) return MPDP_EINVAL;
        if (L.adj[u] & (1u << v)) return MPDP_EINVAL;  // duplicate predicate
        if (!std::isfinite(sel[i]) || !(sel[i] > 0.0) || !(sel[i] <= 1.0)) return MPDP_EINVAL;
        L.adj[u] |= 1u << v;
        L.adj[v] |= 1u << u;
        q.sel_full[u * 32 + v] = sel[i];
        q.sel_full[v * 32 + u] = sel[i];
    }
    // connectivity of the whole join graph (no cross products, Section 2.1.1)
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t nb = 0;
        for (uint32_t t = frontier; t; t &= t - 1) nb |= L.adj[__builtin_ctz(t)];
        frontier = nb & full & ~seen;
        seen |= frontier;
    }
    if (seen != full) return MPDP_ENOTCONNECTED;
    q.is_tree = (m == n - 1);
    g.is_tree = q.is_tree ? 1u : 0u;
    // tree rooted at relation 0: parent bits and subtree sets, via BFS order;
    // flat when every other relation hangs on relation 0 (a star around it)
    g.flat = 0u;
    if (q.is_tree) {
        int order[32], head = 0, tail = 0;
        int parent[32];
        for (int v = 0; v < 32; ++v) parent[v] = -1;
        uint32_t vis = 1u;
        order[tail++] = 0;
        while (head < tail) {
            const int v = order[head++];
            for (uint32_t t = L.adj[v] & ~vis; t; t &= t - 1) {
                const int c = __builtin_ctz(t);
                parent[c] = v;
                vis |= 1u << c;
                order[tail++] = c;
            }
        }
        for (uint32_t v = 0; v < n; ++v) {
            L.pd[v][1] = 1u << v;
            L.pd[v][0] = parent[v] >= 0 ? (1u << parent[v]) : 0u;
        }
        for (int i = tail - 1; i > 0; --i) L.pd[parent[order[i]]][1] |= L.pd[order[i]][1];
        g.flat = (n >= 2 && (L.adj[0] & full) == (full & ~1u)) ? 1u : 0u;
    }
    // selectivities of the edges (u, v), u < v, grouped by v, u ascending
    uint32_t at = 0;
    for (uint32_t v = 0; v < n; ++v) {
        L.selrow[v] = at;
        const uint32_t lower = L.adj[v] & ((1u << v) - 1u);
        L.lo[v][0] = lower & (0u - lower);
        L.lo[v][1] = lower & ~L.lo[v][0];
        L.csel[v][0] = L.card[v];
        L.csel[v][1] = lower ? q.sel_full[__builtin_ctz(lower) * 32 + v] : 1.0;
        for (uint32_t t = lower; t; t &= t - 1)
            L.sel[at++] = q.sel_full[__builtin_ctz(t) * 32 + v];
    }
    for (uint32_t v = n; v < 32; ++v) L.csel[v][0] = L.csel[v][1] = 1.0;
    // byte tables: entry x is entry x without its lowest bit, plus that
    // relation's row (relations beyond n have empty rows)
    uint32_t kids[32] = {0};  // tree joins: children of each relation
    if (q.is_tree)
        for (uint32_t v = 1; v < n; ++v) kids[__builtin_ctz(L.pd[v][0])] |= 1u << v;
    for (int b = 0; b < 4; ++b) {
        L.nb[b][0] = 0;
        L.ch[b][0] = 0;
        for (uint32_t x = 1; x < 256; ++x) {
            const uint32_t v = 8u * b + (uint32_t)__builtin_ctz(x);
            L.nb[b][x] = L.nb[b][x & (x - 1)] | (v < n ? L.adj[v] : 0u);
            L.ch[b][x] = L.ch[b][x & (x - 1)] | kids[v];
        }
    }
    std::memcpy(L.binom, binom_table(), sizeof(L.binom));
    uint64_t off = 0;
    for (uint32_t k = 0; k < 34; ++k) {
        L.loff[k] = off;
        if (k <= n) off += binom64(n, k);
    }
    return MPDP_OK;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

mpdp_status leaf_only(const Query &q, mpdp_plan_node *plan, double *cost_out) {
    plan[0] = mpdp_plan_node{-1, -1, 1u, MPDP_OP_SCAN, q.g.lds.bcost[0], q.g.lds.card[0]};
    *cost_out = q.g.lds.bcost[0];
    return MPDP_OK;
}

#define HIPCHK(expr)                                \
    do {                                            \
        if ((expr) != hipSuccess) return MPDP_EDEVICE; \
    } while (0)

// Pinned host staging of the calling thread, at least `bytes` (kept for the
// process's lifetime; nullptr if pinned memory cannot be had, and the caller
// then copies from pageable memory).
char *pinned_staging(size_t bytes) {
    thread_local char *buf = nullptr;
    thread_local size_t cap = 0;
    if (cap >= bytes) return buf;
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (buf) (void)hipHostFree(buf);
    buf = static_cast<char *>(p);
    cap = bytes;
    return buf;
}

// Bytes of counters, plan and root cost read back per call, as far as the
// no-allocation path keeps them on the stack (n <= 32 needs under 3 KB).
constexpr size_t kNoAllocDownBytes = 4096;

// Device buffer of the unfused-prune ablation (measurement only), one per
// device, grown on demand and kept for the process's lifetime.
void *ablation_buffer(size_t bytes) {
    static std::mutex mu;
    static void *buf[64] = {nullptr};
    static size_t cap[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (cap[dev] < bytes) {
        if (buf[dev]) (void)hipFree(buf[dev]);
        buf[dev] = nullptr;
        cap[dev] = 0;
        if (hipMalloc(&buf[dev], bytes) != hipSuccess) {
            (void)hipGetLastError();
            buf[dev] = nullptr;
            return nullptr;
        }
        cap[dev] = bytes;
    }
    return buf[dev];
}

// A call's launch sequence (upload, init, every level, plan, readback) is
// recorded once per workspace, staging buffer, device and shape into a HIP
// graph and replayed, which takes the host's per-launch work out of the
// call (star 12: 0.122 -> 0.112 ms; the rest is the levels' own latency).
// Calls with timing events or ablation flags launch directly.
#ifndef MPDP_GRAPH_MAX_REL
#define MPDP_GRAPH_MAX_REL 32
#endif
constexpr uint32_t kGraphMaxRel = MPDP_GRAPH_MAX_REL;
constexpr size_t kGraphCacheSize = 32;  // recorded graphs kept per thread

struct GraphKey {
    void *ws, *pin;
    uint32_t n, cost_model;
    bool general, flat;  // the level kernels recorded depend on both
    bool operator==(const GraphKey &o) const {
        return ws == o.ws && pin == o.pin && n == o.n && cost_model == o.cost_model && general == o.general &&
               flat == o.flat;
    }
};

struct GraphEntry {
    GraphKey key;
    int dev;
    hipGraphExec_t exec;
    uint64_t used;
};

// Per thread; entries are destroyed on eviction only (a thread's exit may
// come after the runtime's own teardown).
struct GraphCache {
    std::vector<GraphEntry> entries;
    hipStream_t capture[64] = {nullptr};  // per device, non-blocking, default priority
    uint64_t tick = 0;
};

template <class Enqueue>
hipError_t cached_graph(const GraphKey &key, Enqueue &&enqueue, hipGraphExec_t &out) {
    thread_local GraphCache *cache = new GraphCache();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    for (GraphEntry &g : cache->entries)
        if (g.dev == dev && g.key == key) {
            g.used = ++cache->tick;
            out = g.exec;
            return hipSuccess;
        }
    hipStream_t &cs = cache->capture[dev];
    if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t er = enqueue(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (er != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return er != hipSuccess ? er : e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (cache->entries.size() >= kGraphCacheSize) {
        size_t oldest = 0;
        for (size_t i = 1; i < cache->entries.size(); ++i)
            if (cache->entries[i].used < cache->entries[oldest].used) oldest = i;
        (void)hipGraphExecDestroy(cache->entries[oldest].exec);
        cache->entries.erase(cache->entries.begin() + (long)oldest);
    }
    cache->entries.push_back(GraphEntry{key, dev, exec, ++cache->tick});
    out = exec;
    return hipSuccess;
}

struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipError_t make(size_t k) {
        ev.resize(k, nullptr);
        for (auto &e : ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) { e = nullptr; return r; }
        }
        return hipSuccess;
    }
};

// One exact optimization in the workspace d_ws on stream s.  With
// no_alloc, nothing is allocated on the host or the device: the query
// information goes up and the plan comes back through pageable memory (the
// calling thread's stack), and MPDP_FLAG_TIMING is refused (its events
// would be created here).
mpdp_status run(const Query &q, void *d_ws, size_t ws_bytes, hipStream_t s, uint32_t flags,
                mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out, double t0,
                bool force_general, bool no_alloc = false) {
    const uint32_t n = q.n;
    const Layout L = make_layout(n);
    if (ws_bytes < L.total) return MPDP_ENOMEM;
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return MPDP_EINVAL;
    char *base = static_cast<char *>(d_ws);
    MemoPtrs memo{reinterpret_cast<double *>(base + L.cost), reinterpret_cast<double *>(base + L.card),
                  reinterpret_cast<uint32_t *>(base + L.left), reinterpret_cast<uint8_t *>(base + L.op)};
    uint32_t *list = reinterpret_cast<uint32_t *>(base + L.list);
    uint32_t *heavy = reinterpret_cast<uint32_t *>(base + L.heavy);
    mpdp::HeavyPart *parts = reinterpret_cast<mpdp::HeavyPart *>(base + L.parts);
    DevGraph *dg = reinterpret_cast<DevGraph *>(base + L.graph);
    Counters *cnt = reinterpret_cast<Counters *>(base + L.counters);
    mpdp_plan_node *dplan = reinterpret_cast<mpdp_plan_node *>(base + L.plan);
    double *droot = reinterpret_cast<double *>(base + L.root);

    const bool timing = (flags & MPDP_FLAG_TIMING) != 0;
    if (timing && no_alloc) return MPDP_EINVAL;
    EventPool ev;
    if (timing) HIPCHK(ev.make(4 * (size_t)n));

    DevGraph *hg = const_cast<DevGraph *>(&q.g);
    hg->ablate = (flags & MPDP_FLAG_ABLATE_DPSUB) ? mpdp::kAblateDpsub : 0u;
    // upload and readback go through this thread's pinned staging buffer
    // (plain DMA, no runtime-side staging copy); the call waits for its
    // stream before returning, so the buffer is free again by the next call
    const size_t down_bytes = L.root + sizeof(double) - L.counters;
    alignas(16) char down_stack[kNoAllocDownBytes];
    if (no_alloc && down_bytes > sizeof(down_stack)) return MPDP_ETOOLARGE;
    char *pin = no_alloc ? nullptr : pinned_staging(sizeof(DevGraph) > down_bytes ? sizeof(DevGraph) : down_bytes);
    const bool general = force_general || !q.is_tree;
    // unfused-prune ablation (tree joins): room for every pair key and set
    // record of the widest level
    const bool unfused = !general && (flags & MPDP_FLAG_ABLATE_UNFUSED_PRUNE) != 0;
    mpdp::PairKey *ukeys = nullptr;
    mpdp::PruneRec *urecs = nullptr;
    if (unfused) {
        uint64_t most_keys = 0, most_sets = 0;
        for (uint32_t k = 2; k <= n; ++k) {
            most_keys = std::max<uint64_t>(most_keys, binom64(n, k) * k);
            most_sets = std::max<uint64_t>(most_sets, binom64(n, k));
        }
        const size_t kb = align_up(sizeof(mpdp::PairKey) * most_keys);
        char *ab = static_cast<char *>(ablation_buffer(kb + sizeof(mpdp::PruneRec) * most_sets));
        if (!ab) return MPDP_ENOMEM;
        ukeys = reinterpret_cast<mpdp::PairKey *>(ab);
        urecs = reinterpret_cast<mpdp::PruneRec *>(ab + kb);
    }
    uint64_t candidates = 0;
    uint32_t launches = 0;
    for (uint32_t k = 2; k <= n; ++k) {
        candidates += binom64(n, k);
        ++launches;
    }
    std::vector<char> down_pageable((pin || no_alloc) ? 0 : down_bytes);
    char *down = pin ? pin : (no_alloc ? down_stack : down_pageable.data());
    // the whole call on one stream: upload, init, every level, plan, readback
    auto enqueue = [&](hipStream_t st) -> hipError_t {
        hipError_t e = hipMemcpyAsync(dg, pin ? static_cast<const void *>(pin) : static_cast<const void *>(&q.g),
                                      sizeof(DevGraph), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = mpdp::launch_init(dg, n, memo, cnt, st);
        for (uint32_t k = 2; k <= n && e == hipSuccess; ++k) {
            const uint64_t nc = binom64(n, k);
            if (timing) e = hipEventRecord(ev.ev[4 * k - 8], st);
            if (e == hipSuccess && general) e = mpdp::launch_filter(dg, k, nc, list, cnt, st);
            if (e == hipSuccess && timing) e = hipEventRecord(ev.ev[4 * k - 7], st);
            if (e != hipSuccess) break;
            if (general)
                e = mpdp::launch_eval_general(dg, q.cost_model, k, nc, list, heavy, cnt, memo, parts, st);
            else if (unfused)  // ablation: evaluate writes every pair's key, prune reduces
                e = mpdp::launch_level_tree_unfused(dg, q.cost_model, k, nc, q.g.flat != 0, cnt, memo, ukeys, urecs,
                                                    st);
            else  // tree joins: unrank, filter and evaluate in one kernel per level
                e = mpdp::launch_level_tree(dg, q.cost_model, n, k, nc, (flags & MPDP_FLAG_ABLATE_NO_COMPACTION) == 0,
                                            q.g.flat != 0, cnt, memo, st);
            if (e == hipSuccess && timing) e = hipEventRecord(ev.ev[4 * k - 6], st);
        }
        if (e == hipSuccess) e = mpdp::launch_extract(dg, n, memo, dplan, droot, cnt, st);
        // counters, plan and root cost are adjacent in the workspace: one copy back
        if (e == hipSuccess) e = hipMemcpyAsync(down, cnt, down_bytes, hipMemcpyDeviceToHost, st);
        return e;
    };
    if (pin) std::memcpy(pin, &q.g, sizeof(DevGraph));
    const bool graphed = pin && !timing && flags == 0 && n <= kGraphMaxRel;
    if (graphed) {
        // replay the sequence recorded once for this workspace, staging
        // buffer and shape (the upload reads the staging buffer at replay)
        hipGraphExec_t exec = nullptr;
        HIPCHK(cached_graph(GraphKey{d_ws, pin, n, (uint32_t)q.cost_model, general, q.g.flat != 0}, enqueue, exec));
        HIPCHK(hipGraphLaunch(exec, s));
    } else {
        HIPCHK(enqueue(s));
    }
    HIPCHK(hipStreamSynchronize(s));
    Counters hc;
    std::memcpy(&hc, down, sizeof(Counters));
    if (hc.extract_error) return MPDP_EDEVICE;
    std::memcpy(plan_out, down + (L.plan - L.counters), sizeof(mpdp_plan_node) * (2 * n - 1));
    std::memcpy(cost_out, down + (L.root - L.counters), sizeof(double));
    if (stats_out) {
        mpdp_stats st{};
        st.candidates = candidates;
        uint64_t conn = 0, tree_ccp = 0;
        for (uint32_t k = 2; k <= n; ++k) {
            conn += hc.level_count[k] + hc.general_count[k];
            tree_ccp += (uint64_t)(k - 1) * hc.level_count[k];
        }
        st.connected_sets = conn;
        if (general) {
            st.ccp_pairs = hc.ccp;
            st.evaluated_pairs = hc.evaluated;
        } else {
            st.ccp_pairs = tree_ccp;
            st.evaluated_pairs = 2 * tree_ccp;
        }
        st.levels = n - 1;
        st.eval_launches = launches;
        if (timing) {
            double f = 0.0, e = 0.0;
            for (uint32_t k = 2; k <= n; ++k) {
                float a = 0.f, b = 0.f;
                HIPCHK(hipEventElapsedTime(&a, ev.ev[4 * k - 8], ev.ev[4 * k - 7]));
                HIPCHK(hipEventElapsedTime(&b, ev.ev[4 * k - 7], ev.ev[4 * k - 6]));
                f += a;
                e += b;
            }
            st.ms_filter = f;
            st.ms_eval = e;
        }
        st.ms_total = now_ms() - t0;
        *stats_out = st;
    }
    return MPDP_OK;
}

// Internal flag for tests: run Alg. 3 (the general kernel) on tree joins too.
constexpr uint32_t kFlagForceGeneral = 0x100u;
constexpr uint32_t kFlagBatchAllTeams = 0x200u;  // test aid: every query that may take a team takes the largest

// ---------------------------------------------------------------- batch

struct BatchLayout {
    size_t binom, counters, queries, teams, edges, cards, sels, bcosts, plans, out, slots, slot_bytes, total;
    uint32_t workgroups, maxn, max_teams, max_entries;
    uint64_t sum_m, sum_n, sum_nodes;
};

// Only a large cyclic query may be shared by a team of workgroups (a tree
// query's sets are cheap and fill one workgroup well).  The layout depends
// on the shapes alone, so it leaves room for every such query to take the
// largest team; which ones do is decided per run from their edges.
bool team_eligible(const mpdp_batch_query &Q) { return Q.n >= mpdp::kTeamMinRel && Q.m != Q.n - 1; }

bool batch_layout(uint32_t nq, const mpdp_batch_query *qs, BatchLayout &B) {
    B = BatchLayout{};
    if (nq == 0 || !qs) return false;
    uint32_t maxn = 1;
    for (uint32_t i = 0; i < nq; ++i) {
        if (qs[i].n == 0 || qs[i].n > mpdp::kBatchMaxRel) return false;
        maxn = qs[i].n > maxn ? qs[i].n : maxn;
        B.sum_m += qs[i].m;
        B.sum_n += qs[i].n;
        B.sum_nodes += 2ull * qs[i].n - 1;
    }
    B.maxn = maxn;
    for (uint32_t i = 0; i < nq; ++i) B.max_teams += team_eligible(qs[i]) ? 1u : 0u;
    B.max_entries = nq + (mpdp::kTeamSize - 1) * B.max_teams;
    // every team fits at once: max_entries >= kTeamSize whenever a team may form
    B.workgroups = B.max_entries < mpdp::kBatchWorkgroups ? B.max_entries : mpdp::kBatchWorkgroups;
    size_t o = 0;
    B.binom = o;    o = align_up(o + 33 * 33 * 4);
    B.counters = o; o = align_up(o + sizeof(mpdp::BatchCounters));
    B.queries = o;  o = align_up(o + sizeof(mpdp::BatchQueryDev) * B.max_entries);
    B.teams = o;    o = align_up(o + sizeof(mpdp::TeamRec) * B.max_teams);
    B.edges = o;    o = align_up(o + 8 * B.sum_m);
    B.cards = o;    o = align_up(o + 8 * B.sum_n);
    B.sels = o;     o = align_up(o + 8 * B.sum_m);
    B.bcosts = o;   o = align_up(o + 8 * B.sum_n);
    B.plans = o;    o = align_up(o + sizeof(mpdp_plan_node) * B.sum_nodes);
    B.out = o;      o = align_up(o + sizeof(mpdp::BatchOut) * nq);
    const uint64_t N = 1ull << maxn;
    B.slot_bytes = align_up(21 * N) + align_up(12 * binom64(maxn, maxn / 2));  // memo, two set lists, heavy list
    B.slots = o;    o += B.slot_bytes * B.workgroups;
    B.total = align_up(o);
    return true;
}

// Host validation of one batch query (same rules as mpdp_optimize).
mpdp_status validate_batch_query(const mpdp_batch_query &Q, const mpdp_edge *edges, const double *card,
                                 const double *sel, const double *bcost) {
    const uint32_t n = Q.n, m = Q.m;
    if (n == 0) return MPDP_EINVAL;
    if (n > mpdp::kBatchMaxRel) return MPDP_ETOOLARGE;
    if (m > n * (n - 1) / 2) return MPDP_EINVAL;
    uint32_t adj[32] = {0};
    for (uint32_t v = 0; v < n; ++v) {
        const double c = card[Q.card_offset + v];
        if (!std::isfinite(c) || !(c >= 1.0)) return MPDP_EINVAL;
        if (bcost && (!std::isfinite(bcost[Q.card_offset + v]) || !(bcost[Q.card_offset + v] >= 0.0)))
            return MPDP_EINVAL;
    }
    for (uint32_t i = 0; i < m; ++i) {
        const mpdp_edge e = edges[Q.edge_offset + i];
        const double s = sel[Q.edge_offset + i];
        if (e.u >= n || e.v >= n || e.u == e.v) return MPDP_EINVAL;
        if (adj[e.u] & (1u << e.v)) return MPDP_EINVAL;
        if (!std::isfinite(s) || !(s > 0.0) || !(s <= 1.0)) return MPDP_EINVAL;
        adj[e.u] |= 1u << e.v;
        adj[e.v] |= 1u << e.u;
    }
    const uint32_t full = (1u << n) - 1u;
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t nb = 0;
        for (uint32_t t = frontier; t; t &= t - 1) nb |= adj[__builtin_ctz(t)];
        frontier = nb & full & ~seen;
        seen |= frontier;
    }
    return seen == full ? MPDP_OK : MPDP_ENOTCONNECTED;
}

// Packed per-query schedule of the batched kernel (layout in mpdp_internal.h).
bool encode_schedule(const mpdp_batch_schedule &sc, uint32_t &packed) {
    uint32_t c;
    switch (sc.tree_chunk) {
        case 1: c = 0; break;
        case 2: c = 1; break;
        case 4: c = 2; break;
        default: return false;
    }
    if (sc.heavy_chunks < 1 || sc.heavy_chunks > 0xffffu) return false;
    packed = c | (sc.heavy_chunks << mpdp::kSchedHeavyShift);
    return true;
}

mpdp_status check_batch_args(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                             const double *cardinalities, const double *selectivities, const double *base_costs,
                             mpdp_cost_model cost_model, const mpdp_batch_schedule *sched) {
    if (nq == 0 || !queries || !cardinalities) return MPDP_EINVAL;
    if (cost_model != MPDP_COST_COUT && cost_model != MPDP_COST_PGLIKE) return MPDP_EINVAL;
    uint64_t sum_m = 0;
    for (uint32_t i = 0; i < nq; ++i) sum_m += queries[i].m;
    if (sum_m > 0 && (!edges || !selectivities)) return MPDP_EINVAL;
    for (uint32_t i = 0; i < nq; ++i) {
        const mpdp_status st = validate_batch_query(queries[i], edges, cardinalities, selectivities, base_costs);
        if (st != MPDP_OK) return st;
        uint32_t packed;
        if (sched && !encode_schedule(sched[i], packed)) return MPDP_EINVAL;
    }
    return MPDP_OK;
}

// Predicted device time (ms) of a query alone on one workgroup of the
// batched kernel, for scheduling only.  Its connected sets are counted on a
// breadth-first spanning tree from relation 0 (the subtrees of a rooted
// tree: f(v) = prod over children of (1 + f(child)), summed over v).  A
// tree query's time is close to linear in that count and in n^2; a cyclic
// query's follows a power law in it and in 1 + its extra edges, and grows
// exponentially with the size of
// its 2-core (the relations left after repeatedly removing those of degree
// one), which bounds the blocks Alg. 3 walks.  The coefficients were fitted
// to measured per-query times of mixed batches of 8-20 relations on MI355X.
double predicted_ms(const mpdp_batch_query &Q, const mpdp_edge *edges) {
    const uint32_t n = Q.n;
    uint32_t adj[32] = {0};
    for (uint32_t e = 0; e < Q.m; ++e) {
        const mpdp_edge E = edges[Q.edge_offset + e];
        adj[E.u] |= 1u << E.v;
        adj[E.v] |= 1u << E.u;
    }
    uint32_t order[32], parent[32], head = 0, tail = 0, seen = 1u;
    order[tail++] = 0;
    parent[0] = 0;
    while (head < tail) {
        const uint32_t v = order[head++];
        for (uint32_t T = adj[v] & ~seen; T; T &= T - 1) {
            const uint32_t c = (uint32_t)__builtin_ctz(T);
            seen |= 1u << c;
            parent[c] = v;
            order[tail++] = c;
        }
    }
    double f[32], subtrees = 0.0;
    for (uint32_t i = 0; i < tail; ++i) f[order[i]] = 1.0;
    for (uint32_t i = tail; i-- > 1;) f[parent[order[i]]] *= 1.0 + f[order[i]];
    for (uint32_t i = 0; i < tail; ++i) subtrees += f[order[i]];
    const uint32_t extra = Q.m - (n - 1);
    if (extra == 0) return std::max(0.05, -0.361 + 1.20e-5 * subtrees + 0.00308 * (double)(n * n));
    uint32_t alive = (n == 32) ? ~0u : (1u << n) - 1u;
    for (bool changed = true; changed;) {
        changed = false;
        for (uint32_t T = alive; T; T &= T - 1) {
            const uint32_t v = (uint32_t)__builtin_ctz(T);
            if (__builtin_popcount(adj[v] & alive) <= 1) {
                alive &= ~(1u << v);
                changed = true;
            }
        }
    }
    const double core = (double)__builtin_popcount(alive);
    return std::exp(-6.466 + 0.1238 * core) * std::pow(subtrees, 0.856) * std::pow(1.0 + extra, 0.080);
}

// Team size of a query from its predicted time alone on one workgroup.
uint32_t team_size(const mpdp_batch_query &Q, double ms) {
    if (!team_eligible(Q)) return 1;
    return ms >= 8.0 ? mpdp::kTeamSize : ms >= 3.0 ? mpdp::kTeamSize / 2 : 1u;
}

// Order in which the workgroups take the queries (longest predicted time
// first, ties in input order), each query's team size in that order, and
// each query's first plan node in input order.
void batch_order(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                 std::vector<uint32_t> &order, std::vector<uint32_t> &team, std::vector<uint64_t> &plan_at,
                 bool all_teams = false) {
    std::vector<double> ms(nq);
    for (uint32_t i = 0; i < nq; ++i) ms[i] = predicted_ms(queries[i], edges);
    order.resize(nq);
    for (uint32_t i = 0; i < nq; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return ms[a] > ms[b]; });
    team.resize(nq);
    for (uint32_t j = 0; j < nq; ++j)
        team[j] = all_teams ? (team_eligible(queries[order[j]]) ? mpdp::kTeamSize : 1u)
                            : team_size(queries[order[j]], ms[order[j]]);
    plan_at.resize(nq);
    uint64_t p = 0;
    for (uint32_t i = 0; i < nq; ++i) { plan_at[i] = p; p += 2ull * queries[i].n - 1; }
}

// Host image of everything the batched kernel reads (B.plans bytes), to be
// uploaded to the workspace in one copy.
void fill_batch_upload(char *up, const BatchLayout &B, uint32_t nq, const mpdp_batch_query *queries,
                       const std::vector<uint32_t> &order, const std::vector<uint32_t> &team_of,
                       const std::vector<uint64_t> &plan_at,
                       const mpdp_edge *edges, const double *cardinalities, const double *selectivities,
                       const double *base_costs, mpdp_cost_model cost_model, const mpdp_batch_schedule *sched) {
    std::memset(up, 0, B.plans);
    std::memcpy(up + B.binom, binom_table(), 33 * 33 * sizeof(uint32_t));
    auto *bc = reinterpret_cast<mpdp::BatchCounters *>(up + B.counters);
    bc->next = 0;
    bc->entries = 0;
    bc->t0 = ~0ull;
    auto *dq = reinterpret_cast<mpdp::BatchQueryDev *>(up + B.queries);
    uint32_t *de = reinterpret_cast<uint32_t *>(up + B.edges);
    double *dc = reinterpret_cast<double *>(up + B.cards);
    double *ds = reinterpret_cast<double *>(up + B.sels);
    double *db = reinterpret_cast<double *>(up + B.bcosts);
    uint64_t eo = 0, co = 0;
    uint32_t entry = 0, team_rec = 0;
    for (uint32_t j = 0; j < nq; ++j) {
        const uint32_t i = order[j];
        const mpdp_batch_query &Q = queries[i];
        uint32_t packed = mpdp::kSchedDefault;
        if (sched) (void)encode_schedule(sched[i], packed);  // checked by check_batch_args
        const uint32_t team = team_of[j];
        for (uint32_t member = 0; member < team; ++member)
            dq[entry++] = mpdp::BatchQueryDev{Q.n, Q.m, Q.m == Q.n - 1 ? 1u : 0u, (uint32_t)cost_model,
                                              co, eo, plan_at[i], packed, j, team, member,
                                              team > 1 ? team_rec : 0u, 0u};
        if (team > 1) ++team_rec;
        for (uint32_t v = 0; v < Q.n; ++v) {
            dc[co + v] = cardinalities[Q.card_offset + v];
            db[co + v] = base_costs ? base_costs[Q.card_offset + v] : 0.0;
        }
        for (uint32_t e = 0; e < Q.m; ++e) {
            de[2 * (eo + e)] = edges[Q.edge_offset + e].u;
            de[2 * (eo + e) + 1] = edges[Q.edge_offset + e].v;
            ds[eo + e] = selectivities[Q.edge_offset + e];
        }
        co += Q.n;
        eo += Q.m;
    }
    bc->entries = entry;  // at most B.max_entries: only eligible queries take teams
}

hipError_t enqueue_batch_kernel(char *base, const BatchLayout &B, uint32_t nq, mpdp_cost_model cost_model,
                                bool with_bcosts, hipStream_t s) {
    (void)nq;  // the kernel walks the queue entries, counted in the uploaded counters
    return mpdp::launch_batch(cost_model, B.workgroups, reinterpret_cast<mpdp::BatchQueryDev *>(base + B.queries),
                              reinterpret_cast<uint32_t *>(base + B.edges),
                              reinterpret_cast<double *>(base + B.cards), reinterpret_cast<double *>(base + B.sels),
                              with_bcosts ? reinterpret_cast<double *>(base + B.bcosts) : nullptr,
                              reinterpret_cast<uint32_t *>(base + B.binom), base + B.slots, B.slot_bytes, B.maxn,
                              reinterpret_cast<mpdp_plan_node *>(base + B.plans),
                              reinterpret_cast<mpdp::BatchOut *>(base + B.out),
                              reinterpret_cast<mpdp::TeamRec *>(base + B.teams),
                              reinterpret_cast<mpdp::BatchCounters *>(base + B.counters), s);
}

// Per-query results from the downloaded outputs (outs in workgroup order).
mpdp_status unpack_batch(uint32_t nq, const std::vector<uint32_t> &order, const mpdp::BatchOut *outs,
                         const mpdp::BatchCounters &hbc, int rate_khz, double *costs_out, double *latency_us_out,
                         double *start_us_out, mpdp_batch_stats *st) {
    const double us_per_tick = rate_khz > 0 ? 1e3 / (double)rate_khz : 0.0;
    for (uint32_t j = 0; j < nq; ++j) {
        const mpdp::BatchOut &o = outs[j];
        const uint32_t i = order[j];
        if (o.error) return MPDP_EDEVICE;
        costs_out[i] = o.cost;
        if (latency_us_out) latency_us_out[i] = (double)(o.t_end - hbc.t0) * us_per_tick;
        if (start_us_out) start_us_out[i] = (double)(o.t_start - hbc.t0) * us_per_tick;
        st->connected_sets += o.connected;
        st->ccp_pairs += o.ccp;
        st->evaluated_pairs += o.evaluated;
    }
    return MPDP_OK;
}

int wall_clock_khz() {
    int dev = 0, rate_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return rate_khz;
}

mpdp_status batch_core(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                       const double *cardinalities, const double *selectivities, const double *base_costs,
                       mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes, void *hip_stream,
                       uint32_t flags, const mpdp_batch_schedule *sched, mpdp_plan_node *plans_out,
                       double *costs_out, double *latency_us_out, double *start_us_out,
                       mpdp_batch_stats *stats_out) {
    const double t0 = now_ms();
    if (!plans_out || !costs_out) return MPDP_EINVAL;
    mpdp_status st0 = check_batch_args(nq, queries, edges, cardinalities, selectivities, base_costs, cost_model,
                                       sched);
    if (st0 != MPDP_OK) return st0;
    BatchLayout B;
    if (!batch_layout(nq, queries, B)) return MPDP_EINVAL;
    if (!d_workspace) return MPDP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return MPDP_EINVAL;
    if (ws_bytes < B.total) return MPDP_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char *base = static_cast<char *>(d_workspace);
    std::vector<uint32_t> order, team;
    std::vector<uint64_t> plan_at;
    batch_order(nq, queries, edges, order, team, plan_at, (flags & kFlagBatchAllTeams) != 0);
    std::vector<char> up(B.plans);
    fill_batch_upload(up.data(), B, nq, queries, order, team, plan_at, edges, cardinalities, selectivities, base_costs,
                      cost_model, sched);
    const int rate_khz = wall_clock_khz();
    const bool timing = (flags & MPDP_FLAG_TIMING) != 0;
    EventPool ev;
    if (timing) HIPCHK(ev.make(2));
    HIPCHK(hipMemcpyAsync(base, up.data(), up.size(), hipMemcpyHostToDevice, s));
    if (timing) HIPCHK(hipEventRecord(ev.ev[0], s));
    HIPCHK(enqueue_batch_kernel(base, B, nq, cost_model, base_costs != nullptr, s));
    if (timing) HIPCHK(hipEventRecord(ev.ev[1], s));
    std::vector<mpdp::BatchOut> outs(nq);
    mpdp::BatchCounters hbc{};
    HIPCHK(hipMemcpyAsync(plans_out, base + B.plans, sizeof(mpdp_plan_node) * B.sum_nodes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(outs.data(), base + B.out, sizeof(mpdp::BatchOut) * nq, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hbc, base + B.counters, sizeof(hbc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    mpdp_batch_stats st{};
    const mpdp_status ust = unpack_batch(nq, order, outs.data(), hbc, rate_khz, costs_out, latency_us_out,
                                         start_us_out, &st);
    if (ust != MPDP_OK) return ust;
    if (stats_out) {
        if (timing) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev.ev[0], ev.ev[1]));
            st.ms_kernel = ms;
        }
        st.workgroups = B.workgroups;
        st.max_n = B.maxn;
        st.ms_total = now_ms() - t0;
        *stats_out = st;
    }
    return MPDP_OK;
}

// ---------------------------------------------------------------- batch schedule autotuner

// Class of a query for the autotuner: n, acyclic or not, band of the number
// of edges beyond a spanning tree.
uint32_t tune_class(const mpdp_batch_query &Q) {
    const uint32_t extra = Q.m - (Q.n - 1);  // the join graph is connected: m >= n - 1
    const uint32_t band = extra == 0 ? 0u : (extra <= 2 ? 1u : (extra <= 5 ? 2u : 3u));
    return (Q.n << 2) | band;
}

mpdp_status batch_autotune(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                           const double *card, const double *sel, mpdp_cost_model cm, void *d_ws, size_t ws_bytes,
                           void *stream, uint32_t reps, mpdp_batch_schedule *out, mpdp_batch_tune_stats *stats) {
    const double t0 = now_ms();
    if (!out || reps < 1 || reps > 16) return MPDP_EINVAL;
    mpdp_status st = check_batch_args(nq, queries, edges, card, sel, nullptr, cm, nullptr);
    if (st != MPDP_OK) return st;
    static const uint32_t kTreeCand[] = {4, 2, 1};              // default first
    static const uint32_t kHeavyCand[] = {256, 32, 64, 128, 1024};
    constexpr uint32_t nT = 3, nH = 5, nRuns = 5;
    const mpdp_batch_schedule dflt{4, 256};
    std::vector<uint64_t> nodes(1, 0);
    for (uint32_t i = 0; i < nq; ++i) nodes[0] += 2ull * queries[i].n - 1;
    std::vector<mpdp_plan_node> plans(nodes[0]);
    std::vector<double> costs(nq), lat(nq), start(nq);
    std::vector<mpdp_batch_schedule> sc(nq);
    // times[i][c]: device times of query i under its candidate c
    std::vector<std::vector<double>> times((size_t)nq * 5);
    uint32_t launches = 0;
    for (uint32_t r = 0; r < reps; ++r)
        for (uint32_t run = 0; run < nRuns; ++run) {
            for (uint32_t i = 0; i < nq; ++i) {
                const bool tree = queries[i].m == queries[i].n - 1;
                sc[i] = dflt;
                if (tree) sc[i].tree_chunk = kTreeCand[run < nT ? run : 0];
                else sc[i].heavy_chunks = kHeavyCand[run < nH ? run : 0];
            }
            st = batch_core(nq, queries, edges, card, sel, nullptr, cm, d_ws, ws_bytes, stream, 0, sc.data(),
                            plans.data(), costs.data(), lat.data(), start.data(), nullptr);
            if (st != MPDP_OK) return st;
            ++launches;
            for (uint32_t i = 0; i < nq; ++i) {
                const bool tree = queries[i].m == queries[i].n - 1;
                if (tree ? run >= nT : run >= nH) continue;
                times[(size_t)i * 5 + run].push_back(lat[i] - start[i]);
            }
        }
    // per class and candidate: median over the class's queries and repetitions
    std::vector<uint32_t> cls(nq);
    std::vector<uint32_t> keys;
    for (uint32_t i = 0; i < nq; ++i) {
        cls[i] = tune_class(queries[i]);
        keys.push_back(cls[i]);
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    double est_default = 0.0, est_tuned = 0.0;
    for (uint32_t key : keys) {
        std::vector<uint32_t> members;
        for (uint32_t i = 0; i < nq; ++i)
            if (cls[i] == key) members.push_back(i);
        const bool tree = queries[members[0]].m == queries[members[0]].n - 1;
        const uint32_t ncand = tree ? nT : nH;
        double med[5] = {0, 0, 0, 0, 0};
        for (uint32_t c = 0; c < ncand; ++c) {
            std::vector<double> v;
            for (uint32_t i : members) v.insert(v.end(), times[(size_t)i * 5 + c].begin(), times[(size_t)i * 5 + c].end());
            std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
            med[c] = v[v.size() / 2];
        }
        uint32_t best = 0;  // candidate 0 is the default; a later one must be strictly faster
        for (uint32_t c = 1; c < ncand; ++c)
            if (med[c] < med[best]) best = c;
        for (uint32_t i : members) {
            out[i] = dflt;
            if (tree) out[i].tree_chunk = kTreeCand[best];
            else out[i].heavy_chunks = kHeavyCand[best];
        }
        est_default += med[0] * (double)members.size() * 1e-3;
        est_tuned += med[best] * (double)members.size() * 1e-3;
    }
    if (stats) {
        stats->classes = (uint32_t)keys.size();
        stats->launches = launches;
        stats->est_default_ms = est_default;
        stats->est_tuned_ms = est_tuned;
        stats->ms_total = now_ms() - t0;
    }
    return MPDP_OK;
}

}  // namespace

// ---------------------------------------------------------------- batch captured in a HIP graph

struct mpdp_batch_graph {
    uint32_t nq = 0;
    mpdp_cost_model cm = MPDP_COST_COUT;
    std::vector<mpdp_batch_query> shape;  // n and m per query, offsets as given at creation
    BatchLayout B{};
    std::vector<uint32_t> order, team;    // queue order and team sizes of the current run
    std::vector<uint64_t> plan_at;
    char *base = nullptr;                 // device workspace
    char *h_up = nullptr;                 // pinned: the upload image (B.plans bytes)
    mpdp_plan_node *h_plans = nullptr;    // pinned downloads
    mpdp::BatchOut *h_out = nullptr;
    mpdp::BatchCounters *h_bc = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rate_khz = 0;
};

namespace {

void release_batch_graph(mpdp_batch_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->h_up) (void)hipHostFree(g->h_up);
    if (g->h_plans) (void)hipHostFree(g->h_plans);
    if (g->h_out) (void)hipHostFree(g->h_out);
    if (g->h_bc) (void)hipHostFree(g->h_bc);
    delete g;
}

// Record upload, kernel and downloads on a capture stream of our own (the
// caller's stream may be the legacy default stream, which cannot capture).
mpdp_status capture_batch_graph(mpdp_batch_graph *g) {
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        ok = hipMemcpyAsync(g->base, g->h_up, g->B.plans, hipMemcpyHostToDevice, cs) == hipSuccess &&
             enqueue_batch_kernel(g->base, g->B, g->nq, g->cm, false, cs) == hipSuccess &&
             hipMemcpyAsync(g->h_plans, g->base + g->B.plans, sizeof(mpdp_plan_node) * g->B.sum_nodes,
                            hipMemcpyDeviceToHost, cs) == hipSuccess &&
             hipMemcpyAsync(g->h_out, g->base + g->B.out, sizeof(mpdp::BatchOut) * g->nq, hipMemcpyDeviceToHost,
                            cs) == hipSuccess &&
             hipMemcpyAsync(g->h_bc, g->base + g->B.counters, sizeof(mpdp::BatchCounters), hipMemcpyDeviceToHost,
                            cs) == hipSuccess;
        hipGraph_t graph = nullptr;
        const bool ended = hipStreamEndCapture(cs, &graph) == hipSuccess;
        ok = ok && ended && graph;
        if (graph) g->graph = graph;
    }
    (void)hipStreamDestroy(cs);
    if (!ok) return MPDP_EDEVICE;
    HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    return MPDP_OK;
}

}  // namespace

// ---------------------------------------------------------------- exact step for the large-query heuristics

namespace mpdp_host {

size_t units_workspace_bytes(uint32_t n) { return (n == 0 || n > 32) ? 0 : make_layout(n).total; }

size_t units_batch_workspace_bytes(uint32_t nq, const mpdp_batch_query *queries) {
    BatchLayout B;
    return batch_layout(nq, queries, B) ? B.total : 0;
}

mpdp_status optimize_units(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *card, const double *sel,
                           const double *base_costs, mpdp_cost_model cm, void *d_ws, size_t ws_bytes,
                           hipStream_t s, mpdp_plan_node *plan_out, double *cost_out) {
    const double t0 = now_ms();
    Query q;
    mpdp_status st = validate(n, m, edges, card, sel, cm, base_costs, q);
    if (st != MPDP_OK) return st;
    if (n == 1) return leaf_only(q, plan_out, cost_out);
    return run(q, d_ws, ws_bytes, s, 0, plan_out, cost_out, nullptr, t0, false);
}

size_t noalloc_workspace_bytes(uint32_t n) { return (n == 0 || n > 32) ? 0 : make_layout(n).total; }

const uint32_t *noalloc_setup() { return binom_table(); }

mpdp_status optimize_noalloc(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *card, const double *sel,
                             mpdp_cost_model cm, mpdp_status (*get_ws)(void **), size_t ws_bytes, hipStream_t s,
                             uint32_t flags, mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out) {
    const double t0 = now_ms();
    if (!plan_out || !cost_out) return MPDP_EINVAL;
    if (flags & ~(uint32_t)MPDP_FLAG_ABLATE_NO_COMPACTION & ~(uint32_t)MPDP_FLAG_ABLATE_DPSUB) return MPDP_EINVAL;
    Query q;
    mpdp_status st = validate(n, m, edges, card, sel, cm, nullptr, q);
    if (st != MPDP_OK) return st;
    if (n == 1) {
        st = leaf_only(q, plan_out, cost_out);
        if (stats_out) {
            std::memset(stats_out, 0, sizeof(*stats_out));
            stats_out->ms_total = now_ms() - t0;
        }
        return st;
    }
    if (ws_bytes < make_layout(n).total) return MPDP_ETOOLARGE;
    void *d_ws = nullptr;
    st = get_ws(&d_ws);
    if (st != MPDP_OK) return st;
    return run(q, d_ws, ws_bytes, s, flags, plan_out, cost_out, stats_out, t0,
               (flags & MPDP_FLAG_ABLATE_DPSUB) != 0, true);
}

mpdp_status optimize_units_batch(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                 const double *card, const double *sel, const double *base_costs,
                                 mpdp_cost_model cm, void *d_ws, size_t ws_bytes, hipStream_t s,
                                 mpdp_plan_node *plans_out, double *costs_out) {
    return batch_core(nq, queries, edges, card, sel, base_costs, cm, d_ws, ws_bytes, s, 0, nullptr, plans_out,
                      costs_out, nullptr, nullptr, nullptr);
}

}  // namespace mpdp_host

extern "C" {

size_t mpdp_batch_workspace_bytes(uint32_t nq, const mpdp_batch_query *queries) {
    BatchLayout B;
    return batch_layout(nq, queries, B) ? B.total : 0;
}

mpdp_status mpdp_optimize_batch(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes, void *hip_stream,
                                uint32_t flags, mpdp_plan_node *plans_out, double *costs_out,
                                double *latency_us_out, double *start_us_out, mpdp_batch_stats *stats_out) {
    return batch_core(nq, queries, edges, cardinalities, selectivities, nullptr, cost_model, d_workspace, ws_bytes,
                      hip_stream, flags, nullptr, plans_out, costs_out, latency_us_out, start_us_out, stats_out);
}

mpdp_status mpdp_optimize_batch_sched(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                      const double *cardinalities, const double *selectivities,
                                      mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes,
                                      void *hip_stream, uint32_t flags, const mpdp_batch_schedule *schedules,
                                      mpdp_plan_node *plans_out, double *costs_out, double *latency_us_out,
                                      double *start_us_out, mpdp_batch_stats *stats_out) {
    return batch_core(nq, queries, edges, cardinalities, selectivities, nullptr, cost_model, d_workspace, ws_bytes,
                      hip_stream, flags, schedules, plans_out, costs_out, latency_us_out, start_us_out, stats_out);
}

mpdp_status mpdp_batch_autotune(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes, void *hip_stream,
                                uint32_t reps, mpdp_batch_schedule *schedules_out,
                                mpdp_batch_tune_stats *stats_out) {
    return batch_autotune(nq, queries, edges, cardinalities, selectivities, cost_model, d_workspace, ws_bytes,
                          hip_stream, reps, schedules_out, stats_out);
}

mpdp_status mpdp_batch_graph_create(uint32_t nq, const mpdp_batch_query *queries, mpdp_cost_model cost_model,
                                    void *d_workspace, size_t ws_bytes, mpdp_batch_graph **graph_out) {
    if (!graph_out) return MPDP_EINVAL;
    *graph_out = nullptr;
    if (nq == 0 || !queries) return MPDP_EINVAL;
    if (cost_model != MPDP_COST_COUT && cost_model != MPDP_COST_PGLIKE) return MPDP_EINVAL;
    for (uint32_t i = 0; i < nq; ++i) {
        const mpdp_batch_query &Q = queries[i];
        if (Q.n == 0) return MPDP_EINVAL;
        if (Q.n > mpdp::kBatchMaxRel) return MPDP_ETOOLARGE;
        if (Q.m + 1 < Q.n || Q.m > Q.n * (Q.n - 1) / 2) return MPDP_EINVAL;
    }
    auto *g = new mpdp_batch_graph;
    g->nq = nq;
    g->cm = cost_model;
    g->shape.assign(queries, queries + nq);
    if (!batch_layout(nq, queries, g->B) || !d_workspace ||
        reinterpret_cast<uintptr_t>(d_workspace) % kAlign) {
        release_batch_graph(g);
        return MPDP_EINVAL;
    }
    if (ws_bytes < g->B.total) {
        release_batch_graph(g);
        return MPDP_ENOMEM;
    }
    g->base = static_cast<char *>(d_workspace);
    g->rate_khz = wall_clock_khz();
    const bool ok =
        hipHostMalloc(reinterpret_cast<void **>(&g->h_up), g->B.plans, hipHostMallocDefault) == hipSuccess &&
        hipHostMalloc(reinterpret_cast<void **>(&g->h_plans), sizeof(mpdp_plan_node) * g->B.sum_nodes,
                      hipHostMallocDefault) == hipSuccess &&
        hipHostMalloc(reinterpret_cast<void **>(&g->h_out), sizeof(mpdp::BatchOut) * nq, hipHostMallocDefault) ==
            hipSuccess &&
        hipHostMalloc(reinterpret_cast<void **>(&g->h_bc), sizeof(mpdp::BatchCounters), hipHostMallocDefault) ==
            hipSuccess;
    if (!ok) {
        release_batch_graph(g);
        return MPDP_ENOMEM;
    }
    std::memset(g->h_up, 0, g->B.plans);
    const mpdp_status st = capture_batch_graph(g);
    if (st != MPDP_OK) {
        release_batch_graph(g);
        return st;
    }
    *graph_out = g;
    return MPDP_OK;
}

mpdp_status mpdp_batch_graph_run(mpdp_batch_graph *g, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                 const double *cardinalities, const double *selectivities,
                                 const mpdp_batch_schedule *schedules, void *hip_stream,
                                 mpdp_plan_node *plans_out, double *costs_out, double *latency_us_out,
                                 mpdp_batch_stats *stats_out) {
    const double t0 = now_ms();
    if (!g || !queries || !plans_out || !costs_out) return MPDP_EINVAL;
    for (uint32_t i = 0; i < g->nq; ++i)
        if (queries[i].n != g->shape[i].n || queries[i].m != g->shape[i].m) return MPDP_EINVAL;
    const mpdp_status st0 = check_batch_args(g->nq, queries, edges, cardinalities, selectivities, nullptr, g->cm,
                                             schedules);
    if (st0 != MPDP_OK) return st0;
    // order and teams follow this run's edges; the layout, fixed by the
    // shapes, has room for any choice of teams
    batch_order(g->nq, queries, edges, g->order, g->team, g->plan_at);
    fill_batch_upload(g->h_up, g->B, g->nq, queries, g->order, g->team, g->plan_at, edges, cardinalities, selectivities,
                      nullptr, g->cm, schedules);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIPCHK(hipGraphLaunch(g->exec, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(plans_out, g->h_plans, sizeof(mpdp_plan_node) * g->B.sum_nodes);
    mpdp_batch_stats st{};
    const mpdp_status ust = unpack_batch(g->nq, g->order, g->h_out, *g->h_bc, g->rate_khz, costs_out,
                                         latency_us_out, nullptr, &st);
    if (ust != MPDP_OK) return ust;
    if (stats_out) {
        st.workgroups = g->B.workgroups;
        st.max_n = g->B.maxn;
        st.ms_total = now_ms() - t0;
        *stats_out = st;
    }
    return MPDP_OK;
}

void mpdp_batch_graph_destroy(mpdp_batch_graph *graph) { release_batch_graph(graph); }

const char *mpdp_status_str(mpdp_status s) {
    switch (s) {
        case MPDP_OK: return "ok";
        case MPDP_EINVAL: return "invalid argument";
        case MPDP_ENOTCONNECTED: return "join graph is not connected";
        case MPDP_ETOOLARGE: return "too many relations for this entry point";
        case MPDP_ENOMEM: return "workspace too small or device allocation failed";
        case MPDP_EDEVICE: return "HIP runtime error";
        case MPDP_ETIMEOUT: return "time budget exhausted (the plan found so far was returned)";
    }
    return "unknown status";
}

size_t mpdp_workspace_bytes(uint32_t n, mpdp_cost_model cost_model) {
    (void)cost_model;
    if (n == 0 || n > 32) return 0;
    return make_layout(n).total;
}

mpdp_status mpdp_memo_layout(uint32_t n, size_t *off_cost, size_t *off_card, size_t *off_left, size_t *off_op) {
    if (n == 0 || n > 32 || !off_cost || !off_card || !off_left || !off_op) return MPDP_EINVAL;
    const Layout L = make_layout(n);
    *off_cost = L.cost;
    *off_card = L.card;
    *off_left = L.left;
    *off_op = L.op;
    return MPDP_OK;
}

mpdp_status mpdp_optimize_ws(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *cardinalities,
                             const double *selectivities, mpdp_cost_model cost_model, void *d_workspace,
                             size_t ws_bytes, void *hip_stream, uint32_t flags, mpdp_plan_node *plan_out,
                             double *cost_out, mpdp_stats *stats_out) {
    const double t0 = now_ms();
    if (!plan_out || !cost_out) return MPDP_EINVAL;
    Query q;
    mpdp_status st = validate(n, m, edges, cardinalities, selectivities, cost_model, nullptr, q);
    if (st != MPDP_OK) return st;
    if (n == 1) {
        st = leaf_only(q, plan_out, cost_out);
        if (stats_out) {
            std::memset(stats_out, 0, sizeof(*stats_out));
            stats_out->ms_total = now_ms() - t0;
        }
        return st;
    }
    if (!d_workspace) return MPDP_EINVAL;
    return run(q, d_workspace, ws_bytes, static_cast<hipStream_t>(hip_stream), flags, plan_out, cost_out,
               stats_out, t0, (flags & (kFlagForceGeneral | MPDP_FLAG_ABLATE_DPSUB)) != 0);
}

mpdp_status mpdp_optimize_units(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *cardinalities,
                                const double *selectivities, const double *base_costs, mpdp_cost_model cost_model,
                                void *d_workspace, size_t ws_bytes, void *hip_stream, uint32_t flags,
                                mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out) {
    const double t0 = now_ms();
    if (!plan_out || !cost_out || !base_costs) return MPDP_EINVAL;
    Query q;
    mpdp_status st = validate(n, m, edges, cardinalities, selectivities, cost_model, base_costs, q);
    if (st != MPDP_OK) return st;
    if (n == 1) {
        st = leaf_only(q, plan_out, cost_out);
        if (stats_out) {
            std::memset(stats_out, 0, sizeof(*stats_out));
            stats_out->ms_total = now_ms() - t0;
        }
        return st;
    }
    if (!d_workspace) return MPDP_EINVAL;
    return run(q, d_workspace, ws_bytes, static_cast<hipStream_t>(hip_stream), flags, plan_out, cost_out,
               stats_out, t0, false);
}

mpdp_status mpdp_optimize(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *cardinalities,
                          const double *selectivities, mpdp_cost_model cost_model, mpdp_plan_node *plan_out,
                          double *cost_out, mpdp_stats *stats_out) {
    const double t0 = now_ms();
    if (!plan_out || !cost_out) return MPDP_EINVAL;
    Query q;
    mpdp_status st = validate(n, m, edges, cardinalities, selectivities, cost_model, nullptr, q);
    if (st != MPDP_OK) return st;
    if (n == 1) {
        st = leaf_only(q, plan_out, cost_out);
        if (stats_out) {
            std::memset(stats_out, 0, sizeof(*stats_out));
            stats_out->ms_total = now_ms() - t0;
        }
        return st;
    }
    const size_t bytes = make_layout(n).total;
    void *ws = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess || !ws) {
        (void)hipGetLastError();
        return MPDP_ENOMEM;
    }
    st = run(q, ws, bytes, nullptr, 0, plan_out, cost_out, stats_out, t0, false);
    if (hipFree(ws) != hipSuccess && st == MPDP_OK) st = MPDP_EDEVICE;
    return st;
}

}  // extern "C"
