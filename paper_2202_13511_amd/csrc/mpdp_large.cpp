// Large-query heuristics of Section 4 on the host, with this library's
// exact DP on the GPU as the inner step: GOO, IDP2 with GOO's plan as its
// start (Section 4.1) and UnionDP (Section 4.2, Alg. 4).  The conventions
// the paper leaves open (card of large sets, re-costing, units, tie-breaks,
// the union order) are stated at mpdp_optimize_large in include/mpdp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <queue>
#include <set>
#include <tuple>
#include <unordered_set>
#include <vector>

#include "mpdp.h"
#include "mpdp_host_internal.h"
#include "mpdp_scorer.h"

namespace {

constexpr uint32_t kLargeMaxRel = 4096;
constexpr uint32_t kLargeMaxK = 25;
constexpr uint32_t kBatchUnits = 20;  // parts of at most this many units go through the batched kernel
constexpr bool kOnePerPass = true;    // learned partition: one join (the best-scored) per pass

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- relation sets of any size

struct Bits {
    std::vector<uint64_t> w;
    Bits() = default;
    explicit Bits(size_t words) : w(words, 0ull) {}
    void set(uint32_t v) { w[v >> 6] |= 1ull << (v & 63u); }
    bool has(uint32_t v) const { return (w[v >> 6] >> (v & 63u)) & 1ull; }
    Bits operator|(const Bits &o) const {
        Bits r(w.size());
        for (size_t i = 0; i < w.size(); ++i) r.w[i] = w[i] | o.w[i];
        return r;
    }
    uint32_t lowest() const {
        for (size_t i = 0; i < w.size(); ++i)
            if (w[i]) return (uint32_t)(64 * i + __builtin_ctzll(w[i]));
        return ~0u;
    }
    uint32_t count() const {
        uint32_t c = 0;
        for (uint64_t x : w) c += (uint32_t)__builtin_popcountll(x);
        return c;
    }
    template <class F>
    void each(F f) const {  // ascending
        for (size_t i = 0; i < w.size(); ++i)
            for (uint64_t x = w[i]; x; x &= x - 1) f((uint32_t)(64 * i + __builtin_ctzll(x)));
    }
};

// a < b as binary numbers
bool bits_less(const Bits &a, const Bits &b) {
    for (size_t i = a.w.size(); i-- > 0;)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
    return false;
}

// ---------------------------------------------------------------- query

struct Graph {
    uint32_t n = 0, words = 0;
    int cm = 0;
    std::vector<double> card;
    std::vector<uint32_t> eu, ev;  // edge list order
    std::vector<double> sel;
    std::vector<std::vector<std::pair<uint32_t, double>>> lower;  // per v: (u, sel) of edges (u, v), u < v, u ascending
    std::vector<std::vector<uint32_t>> adj;

    Bits single(uint32_t v) const {
        Bits b(words);
        b.set(v);
        return b;
    }
    // card(S): the canonical product of the exact DP, for a set of any size
    double card_of(const Bits &S) const {
        double c = 1.0;
        S.each([&](uint32_t v) {
            c = c * card[v];
            for (const auto &us : lower[v])
                if (S.has(us.first)) c = c * us.second;
        });
        return c < 1.0 ? 1.0 : c;
    }
    double scan_cost(uint32_t v) const { return cm == MPDP_COST_PGLIKE ? 0.01 * card[v] : 0.0; }
};

// ---------------------------------------------------------------- plans and their re-costing

struct PNode {
    int a = -1, b = -1;  // join children, or -1
    int leaf = -1;       // relation of a leaf
    bool done = false;   // re-costed
    Bits rels;
    double cost = 0.0, card = 0.0;
    uint32_t op = MPDP_OP_SCAN;
    int l = -1, r = -1;  // chosen orientation
};

struct Side {
    const Bits *rels;
    double cost, card;
};

// One join of the re-costing: cheaper orientation and operator; key (cost,
// left relation set as a binary number, HASH before NESTLOOP).
void combine(int cm, const Side &a, const Side &b, double cS, double &cost, uint32_t &op, bool &a_left) {
    const double base = a.cost + b.cost;
    if (cm == MPDP_COST_COUT) {
        cost = base + cS;
        op = MPDP_OP_JOIN;
        a_left = bits_less(*a.rels, *b.rels);
        return;
    }
    const double out = 0.01 * cS;
    double c[2];
    uint32_t o[2];
    const Side *L[2] = {&a, &b}, *R[2] = {&b, &a};
    for (int i = 0; i < 2; ++i) {
        const double hj = ((base + 0.0125 * R[i]->card) + 0.0025 * L[i]->card) + out;
        const double nl = (base + (0.0025 * L[i]->card) * R[i]->card) + out;
        if (hj <= nl) { c[i] = hj; o[i] = MPDP_OP_HASH; }
        else { c[i] = nl; o[i] = MPDP_OP_NESTLOOP; }
    }
    bool first;
    if (c[0] != c[1]) first = c[0] < c[1];
    else first = bits_less(*a.rels, *b.rels);  // the two left sets differ: op is not reached
    cost = first ? c[0] : c[1];
    op = first ? o[0] : o[1];
    a_left = first;
}

struct Pool {
    const Graph *G;
    std::vector<PNode> nodes;
    std::vector<int> leaf_of;

    int leaf(uint32_t v) {
        if (leaf_of[v] >= 0) return leaf_of[v];
        PNode p;
        p.leaf = (int)v;
        nodes.push_back(std::move(p));
        return leaf_of[v] = (int)nodes.size() - 1;
    }
    int join(int a, int b) {
        PNode p;
        p.a = a;
        p.b = b;
        nodes.push_back(std::move(p));
        return (int)nodes.size() - 1;
    }
    // bottom-up re-costing over the base relations, memoised per node
    void recost(int id) {
        // explicit post-order: trees may be as deep as they are wide
        std::vector<std::pair<int, bool>> st{{id, false}};
        while (!st.empty()) {
            auto [x, expanded] = st.back();
            st.pop_back();
            PNode &p = nodes[x];
            if (p.done) continue;
            if (p.leaf >= 0) {
                p.rels = G->single((uint32_t)p.leaf);
                p.cost = G->scan_cost((uint32_t)p.leaf);
                p.card = G->card[p.leaf];
                p.op = MPDP_OP_SCAN;
                p.done = true;
                continue;
            }
            if (!expanded) {
                st.push_back({x, true});
                st.push_back({p.b, false});
                st.push_back({p.a, false});
                continue;
            }
            const PNode &A = nodes[p.a], &B = nodes[p.b];
            Bits S = A.rels | B.rels;
            const double cS = G->card_of(S);
            double cost;
            uint32_t op;
            bool a_left;
            combine(G->cm, Side{&A.rels, A.cost, A.card}, Side{&B.rels, B.cost, B.card}, cS, cost, op, a_left);
            PNode &q = nodes[x];  // (no reallocation happens inside this loop)
            q.rels = std::move(S);
            q.card = cS;
            q.cost = cost;
            q.op = op;
            q.l = a_left ? q.a : q.b;
            q.r = a_left ? q.b : q.a;
            q.done = true;
        }
    }
};

// ---------------------------------------------------------------- exact step on units

struct Unit {
    Bits rels;
    int plan;
    uint32_t low;
};

struct ExactCtx {
    const Graph *G;
    Pool *P;
    hipStream_t s;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<int> where;  // relation -> local unit index, -1 outside
    mpdp_large_stats st{};
    // time budget: wall clock of the call's start and its limit (0: none)
    double t0 = 0.0, budget_ms = 0.0;
    bool over_budget() const { return budget_ms > 0.0 && now_ms() - t0 >= budget_ms; }
    // learned union order: scorer parameters (device) and scratch
    const void *scorer = nullptr;
    void *sc_buf = nullptr;
    size_t sc_bytes = 0;
    // training examples: optimal plan's relation sets and the output
    const std::unordered_set<uint32_t> *plan_sets = nullptr;  // teacher labels (n <= 32)
    bool teacher = false;                                     // score = +1 for plan nodes, -1 otherwise
    std::vector<uint16_t> *ex_x = nullptr;
    std::vector<float> *ex_y = nullptr;

    ~ExactCtx() {
        if (ws) (void)hipFree(ws);
        if (sc_buf) (void)hipFree(sc_buf);
    }
    mpdp_status reserve(size_t bytes) {
        if (bytes <= ws_bytes) return MPDP_OK;
        if (ws) {
            if (hipFree(ws) != hipSuccess) return MPDP_EDEVICE;
            ws = nullptr;
            ws_bytes = 0;
        }
        if (hipMalloc(&ws, bytes) != hipSuccess || !ws) {
            (void)hipGetLastError();
            ws = nullptr;
            return MPDP_ENOMEM;
        }
        ws_bytes = bytes;
        return MPDP_OK;
    }
};

struct UnitQuery {
    std::vector<const Unit *> us;  // labelled by lowest relation
    std::vector<mpdp_edge> edges;
    std::vector<double> card, sel, bcost;
};

void build_unit_query(ExactCtx &X, const std::vector<const Unit *> &units, UnitQuery &Q) {
    const Graph &G = *X.G;
    Q.us = units;
    std::sort(Q.us.begin(), Q.us.end(), [](const Unit *a, const Unit *b) { return a->low < b->low; });
    for (size_t i = 0; i < Q.us.size(); ++i) Q.us[i]->rels.each([&](uint32_t v) { X.where[v] = (int)i; });
    std::map<std::pair<uint32_t, uint32_t>, double> cross;
    for (size_t e = 0; e < G.eu.size(); ++e) {
        const int a = X.where[G.eu[e]], b = X.where[G.ev[e]];
        if (a < 0 || b < 0 || a == b) continue;
        const auto key = std::make_pair((uint32_t)std::min(a, b), (uint32_t)std::max(a, b));
        auto it = cross.find(key);
        if (it == cross.end()) cross.emplace(key, 1.0 * G.sel[e]);
        else it->second = it->second * G.sel[e];
    }
    for (const auto &kv : cross) {
        Q.edges.push_back(mpdp_edge{kv.first.first, kv.first.second});
        Q.sel.push_back(kv.second < DBL_MIN ? DBL_MIN : kv.second);
    }
    for (const Unit *u : Q.us) {
        Q.card.push_back(G.card_of(u->rels));
        X.P->recost(u->plan);
        Q.bcost.push_back(X.P->nodes[u->plan].cost);
    }
    for (const Unit *u : Q.us) u->rels.each([&](uint32_t v) { X.where[v] = -1; });
}

// The DP's plan over units, rebuilt as a plan over base relations.
int plan_from_units(Pool &P, const UnitQuery &Q, const mpdp_plan_node *plan) {
    const uint32_t j = (uint32_t)Q.us.size();
    std::vector<int> id(2 * j - 1);
    for (uint32_t i = 0; i < j; ++i) id[i] = Q.us[i]->plan;
    for (uint32_t i = j; i < 2 * j - 1; ++i) id[i] = P.join(id[plan[i].left], id[plan[i].right]);
    return id[2 * j - 2];
}

// Plan each group of units exactly; returns the new plans in group order.
mpdp_status exact_groups(ExactCtx &X, const std::vector<std::vector<const Unit *>> &groups, std::vector<int> &out) {
    out.assign(groups.size(), -1);
    std::vector<UnitQuery> qs(groups.size());
    std::vector<size_t> todo_batch, todo_single;
    for (size_t g = 0; g < groups.size(); ++g) {
        if (groups[g].size() == 1) {
            out[g] = groups[g][0]->plan;
            continue;
        }
        build_unit_query(X, groups[g], qs[g]);
        X.st.exact_calls += 1;
        X.st.exact_units += groups[g].size();
        X.st.max_units = std::max<uint32_t>(X.st.max_units, (uint32_t)groups[g].size());
        if (groups[g].size() <= kBatchUnits) todo_batch.push_back(g);
        else todo_single.push_back(g);
    }
    const double t0 = now_ms();
    const mpdp_cost_model cm = (mpdp_cost_model)X.G->cm;
    if (todo_batch.size() == 1) todo_single.insert(todo_single.begin(), todo_batch[0]), todo_batch.clear();
    if (!todo_batch.empty()) {
        std::vector<mpdp_batch_query> bq;
        std::vector<mpdp_edge> e;
        std::vector<double> c, s, b;
        uint64_t nodes = 0;
        for (size_t g : todo_batch) {
            const UnitQuery &Q = qs[g];
            bq.push_back(mpdp_batch_query{(uint32_t)Q.us.size(), (uint32_t)Q.edges.size(), (uint32_t)c.size(),
                                          (uint32_t)e.size()});
            e.insert(e.end(), Q.edges.begin(), Q.edges.end());
            s.insert(s.end(), Q.sel.begin(), Q.sel.end());
            c.insert(c.end(), Q.card.begin(), Q.card.end());
            b.insert(b.end(), Q.bcost.begin(), Q.bcost.end());
            nodes += 2 * Q.us.size() - 1;
        }
        const size_t bytes = mpdp_host::units_batch_workspace_bytes((uint32_t)bq.size(), bq.data());
        if (bytes == 0) return MPDP_EINVAL;
        mpdp_status st = X.reserve(bytes);
        if (st != MPDP_OK) return st;
        std::vector<mpdp_plan_node> plans(nodes);
        std::vector<double> costs(bq.size());
        st = mpdp_host::optimize_units_batch((uint32_t)bq.size(), bq.data(), e.data(), c.data(), s.data(), b.data(),
                                             cm, X.ws, X.ws_bytes, X.s, plans.data(), costs.data());
        if (st != MPDP_OK) return st;
        X.st.launches += 1;
        uint64_t at = 0;
        for (size_t g : todo_batch) {
            out[g] = plan_from_units(*X.P, qs[g], plans.data() + at);
            at += 2 * qs[g].us.size() - 1;
        }
    }
    for (size_t g : todo_single) {
        const UnitQuery &Q = qs[g];
        const uint32_t j = (uint32_t)Q.us.size();
        mpdp_status st = X.reserve(mpdp_host::units_workspace_bytes(j));
        if (st != MPDP_OK) return st;
        std::vector<mpdp_plan_node> plan(2 * j - 1);
        double cost = 0.0;
        st = mpdp_host::optimize_units(j, (uint32_t)Q.edges.size(), Q.edges.data(), Q.card.data(), Q.sel.data(),
                                       Q.bcost.data(), cm, X.ws, X.ws_bytes, X.s, plan.data(), &cost);
        if (st != MPDP_OK) return st;
        X.st.launches += 1;
        out[g] = plan_from_units(*X.P, Q, plan.data());
    }
    X.st.ms_exact += now_ms() - t0;
    return MPDP_OK;
}

// ---------------------------------------------------------------- GOO

// GOO from a list of starting trees (relation sets with their plans, in
// order of their lowest relation): join the two adjacent trees whose union
// has the smallest card (ties: the smaller tree indices) until one is left.
int goo_from(const Graph &G, Pool &P, const std::vector<Bits> &rels, const std::vector<int> &plans,
             const std::vector<int> &where) {
    struct Tree {
        Bits rels;
        int plan;
        uint32_t version;
        std::set<uint32_t> nbrs;
        bool alive;
    };
    const uint32_t nt = (uint32_t)rels.size();
    std::vector<Tree> T(nt);
    uint32_t version = 0;
    for (uint32_t t = 0; t < nt; ++t) T[t] = Tree{rels[t], plans[t], version++, {}, true};
    std::set<std::pair<uint32_t, uint32_t>> tedges;
    for (size_t e = 0; e < G.eu.size(); ++e) {
        const uint32_t a = (uint32_t)where[G.eu[e]], b = (uint32_t)where[G.ev[e]];
        if (a == b) continue;
        T[a].nbrs.insert(b);
        T[b].nbrs.insert(a);
        tedges.insert({std::min(a, b), std::max(a, b)});
    }
    using Cand = std::tuple<double, uint32_t, uint32_t, uint32_t, uint32_t>;  // card, i, j, ver i, ver j
    std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> heap;
    for (const auto &[i, j] : tedges)
        heap.push(Cand{G.card_of(T[i].rels | T[j].rels), i, j, T[i].version, T[j].version});
    uint32_t left = nt;
    int root = nt == 1 ? T[0].plan : -1;
    while (left > 1 && !heap.empty()) {
        const auto [c, i, j, vi, vj] = heap.top();
        heap.pop();
        (void)c;
        if (!T[i].alive || !T[j].alive || T[i].version != vi || T[j].version != vj) continue;
        Tree &A = T[i];
        Tree &B = T[j];
        A.rels = A.rels | B.rels;
        A.plan = P.join(A.plan, B.plan);
        A.version = version++;
        B.alive = false;
        std::set<uint32_t> nb;
        for (uint32_t x : A.nbrs) if (x != i && x != j) nb.insert(x);
        for (uint32_t x : B.nbrs) if (x != i && x != j) nb.insert(x);
        A.nbrs = nb;
        B.nbrs.clear();
        for (uint32_t x : nb) {
            T[x].nbrs.erase(j);
            T[x].nbrs.insert(i);
            const uint32_t lo = std::min(i, x), hi = std::max(i, x);
            heap.push(Cand{G.card_of(A.rels | T[x].rels), lo, hi, T[lo].version, T[hi].version});
        }
        --left;
        root = A.plan;
    }
    return left == 1 ? root : -1;
}

int goo(const Graph &G, Pool &P) {
    std::vector<Bits> rels;
    std::vector<int> plans, where(G.n);
    for (uint32_t v = 0; v < G.n; ++v) {
        rels.push_back(G.single(v));
        plans.push_back(P.leaf(v));
        where[v] = (int)v;
    }
    return goo_from(G, P, rels, plans, where);
}

// GOO over the current units of a budgeted run that has run out of time.
int goo_units(const Graph &G, Pool &P, std::vector<Unit> units) {
    std::sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.low < b.low; });
    std::vector<Bits> rels;
    std::vector<int> plans, where(G.n, -1);
    for (size_t i = 0; i < units.size(); ++i) {
        rels.push_back(units[i].rels);
        plans.push_back(units[i].plan);
        units[i].rels.each([&](uint32_t v) { where[v] = (int)i; });
    }
    return goo_from(G, P, rels, plans, where);
}

// ---------------------------------------------------------------- IDP2

mpdp_status idp2(ExactCtx &X, int start, uint32_t k, int &result) {
    const Graph &G = *X.G;
    Pool &P = *X.P;
    struct TNode {
        int l = -1, r = -1;
        int unit = -1;
        // per iteration
        uint32_t cnt = 0, low = 0;
        double cost = 0.0, card = 0.0;
        Bits rels;
        bool card_done = false;
    };
    std::vector<Unit> units;
    std::vector<TNode> T;
    // the start plan as a tree whose leaves are units (one per relation)
    std::function<int(int)> conv = [&](int pid) -> int {
        const PNode &p = P.nodes[pid];
        TNode t;
        if (p.leaf >= 0) {
            units.push_back(Unit{G.single((uint32_t)p.leaf), pid, (uint32_t)p.leaf});
            t.unit = (int)units.size() - 1;
            T.push_back(t);
            return (int)T.size() - 1;
        }
        const int a = conv(p.a);
        const int b = conv(p.b);
        t.l = a;
        t.r = b;
        T.push_back(t);
        return (int)T.size() - 1;
    };
    const int root = conv(start);
    while (T[root].unit < 0) {
        if (X.over_budget()) {
            // anytime: the start tree with the subtrees re-planned so far
            std::function<int(int)> plan_of = [&](int x) -> int {
                if (T[x].unit >= 0) return units[T[x].unit].plan;
                const int a = plan_of(T[x].l);
                return P.join(a, plan_of(T[x].r));
            };
            result = plan_of(root);
            return MPDP_ETIMEOUT;
        }
        X.st.rounds += 1;
        // post-order: units below, relation set, cost (re-costing from the children)
        int best = -1;
        double best_cost = 0.0;
        uint32_t best_low = 0;
        std::vector<std::pair<int, bool>> st{{root, false}};
        while (!st.empty()) {
            auto [x, expanded] = st.back();
            st.pop_back();
            TNode &t = T[x];
            if (t.unit >= 0) {
                const Unit &u = units[t.unit];
                P.recost(u.plan);
                t.cnt = 1;
                t.low = u.low;
                t.rels = u.rels;
                t.cost = P.nodes[u.plan].cost;
                t.card = P.nodes[u.plan].card;
                continue;
            }
            if (!expanded) {
                st.push_back({x, true});
                st.push_back({t.r, false});
                st.push_back({t.l, false});
                continue;
            }
            const TNode &A = T[t.l], &B = T[t.r];
            t.cnt = A.cnt + B.cnt;
            t.low = std::min(A.low, B.low);
            t.rels = A.rels | B.rels;
            if (!t.card_done) {
                t.card = G.card_of(t.rels);
                t.card_done = true;
            }
            uint32_t op;
            bool a_left;
            combine(G.cm, Side{&A.rels, A.cost, A.card}, Side{&B.rels, B.cost, B.card}, t.card, t.cost, op, a_left);
            if (t.cnt >= 2 && t.cnt <= k) {
                // highest cost; ties to the lower lowest relation; first in post-order
                if (best < 0 || t.cost > best_cost || (t.cost == best_cost && t.low < best_low)) {
                    best = x;
                    best_cost = t.cost;
                    best_low = t.low;
                }
            }
        }
        // the units below the picked subtree, re-planned exactly
        std::vector<const Unit *> us;
        std::vector<int> stack{best};
        while (!stack.empty()) {
            const int x = stack.back();
            stack.pop_back();
            if (T[x].unit >= 0) us.push_back(&units[T[x].unit]);
            else { stack.push_back(T[x].r); stack.push_back(T[x].l); }
        }
        std::vector<int> plans;
        mpdp_status s = exact_groups(X, {us}, plans);
        if (s != MPDP_OK) return s;
        Bits rels = T[best].rels;
        const uint32_t low = T[best].low;
        units.push_back(Unit{std::move(rels), plans[0], low});
        T[best].unit = (int)units.size() - 1;
        T[best].l = T[best].r = -1;
    }
    result = units[T[root].unit].plan;
    return MPDP_OK;
}

// ---------------------------------------------------------------- learned union order

uint16_t bf16_bits(double x) {
    const float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Features of candidate unions of two parts (parts: unit indices; pairs
// (a, b), a < b), float64, rounded to float32 and then to bfloat16.  For
// parts A, B with weight w = card(A u B), every pair put as (smaller, larger):
//  0,1 log10 card(A), card(B) / 8;  2 log10 w / 8;
//  3 (log10 w - log10 card(A) - log10 card(B)) / 8;
//  4,5 log10(1 + summed plan cost of the units of A, B) / 8;
//  6,7 log2 relations of A, B / 4;  8,9 candidate unions of A, B / 8;
//  10,11 units of A, B / 8;  12,13 share of A's (B's) candidates with a smaller weight;
//  14,15 log10 w - log10 of the smallest weight at A (B), / 8;
//  16 log2 parts / 12;  17 share of all candidates with a smaller weight;  18 one.
void part_features(const Graph &G, Pool &P, const std::vector<Unit> &units,
                   const std::vector<std::vector<uint32_t>> &parts,
                   const std::vector<std::pair<uint32_t, uint32_t>> &pairs, std::vector<Bits> &rels,
                   std::vector<uint16_t> &X) {
    const size_t np = parts.size(), ne = pairs.size();
    rels.assign(np, Bits(G.words));
    std::vector<double> card(np), cost(np), nrel(np), ucost(units.size());
    for (size_t u = 0; u < units.size(); ++u) {
        P.recost(units[u].plan);
        ucost[u] = P.nodes[units[u].plan].cost;
    }
    for (size_t a = 0; a < np; ++a) {
        double c = 0.0;
        for (uint32_t u : parts[a]) {
            rels[a] = rels[a] | units[u].rels;
            c = c + ucost[u];
        }
        cost[a] = c;
        card[a] = G.card_of(rels[a]);
        nrel[a] = (double)rels[a].count();
    }
    std::vector<double> w(ne);
    std::vector<std::vector<double>> inc(np);
    for (size_t e = 0; e < ne; ++e) {
        w[e] = G.card_of(rels[pairs[e].first] | rels[pairs[e].second]);
        inc[pairs[e].first].push_back(w[e]);
        inc[pairs[e].second].push_back(w[e]);
    }
    X.assign(ne * MPDP_SCORER_IN, 0);
    // candidates with a smaller weight than each: its place among them sorted
    std::vector<double> wsorted(w);
    std::sort(wsorted.begin(), wsorted.end());
    for (size_t e = 0; e < ne; ++e) {
        const uint32_t a = pairs[e].first, b = pairs[e].second;
        double f[MPDP_SCORER_IN] = {0.0};
        const double lw = std::log10(w[e]);
        const double la = std::log10(card[a]), lb = std::log10(card[b]);
        const double pa = std::log10(1.0 + cost[a]), pb = std::log10(1.0 + cost[b]);
        const double na = std::log2(nrel[a]), nb = std::log2(nrel[b]);
        const double da = (double)inc[a].size(), db = (double)inc[b].size();
        const double ua = (double)parts[a].size(), ub = (double)parts[b].size();
        double ca = 0.0, cb = 0.0, cg = 0.0;
        for (double x : inc[a]) ca += x < w[e] ? 1.0 : 0.0;
        for (double x : inc[b]) cb += x < w[e] ? 1.0 : 0.0;
        cg = (double)(std::lower_bound(wsorted.begin(), wsorted.end(), w[e]) - wsorted.begin());
        const double ra = ca / da, rb = cb / db;
        const double ma = lw - std::log10(*std::min_element(inc[a].begin(), inc[a].end()));
        const double mb = lw - std::log10(*std::min_element(inc[b].begin(), inc[b].end()));
        f[0] = std::min(la, lb) / 8; f[1] = std::max(la, lb) / 8;
        f[2] = lw / 8;
        f[3] = (lw - la - lb) / 8;
        f[4] = std::min(pa, pb) / 8; f[5] = std::max(pa, pb) / 8;
        f[6] = std::min(na, nb) / 4; f[7] = std::max(na, nb) / 4;
        f[8] = std::min(da, db) / 8; f[9] = std::max(da, db) / 8;
        f[10] = std::min(ua, ub) / 8; f[11] = std::max(ua, ub) / 8;
        f[12] = std::min(ra, rb); f[13] = std::max(ra, rb);
        f[14] = std::min(ma, mb) / 8; f[15] = std::max(ma, mb) / 8;
        f[16] = std::log2((double)np) / 12;
        f[17] = cg / (double)ne;
        f[18] = 1.0;
        for (int t = 0; t < MPDP_SCORER_IN; ++t) X[e * MPDP_SCORER_IN + t] = bf16_bits(f[t]);
    }
}

// Logits of the rows of X from the scorer on the GPU.
mpdp_status score_rows(ExactCtx &X, const std::vector<uint16_t> &feat, std::vector<float> &logit) {
    const uint32_t rows = (uint32_t)(feat.size() / MPDP_SCORER_IN);
    logit.assign(rows, 0.f);
    if (rows == 0) return MPDP_OK;
    const size_t xb = (2 * feat.size() + 255) & ~(size_t)255, lb = (4 * (size_t)rows + 255) & ~(size_t)255;
    const size_t wb = mpdp_scorer_work_bytes(rows);
    const size_t need = xb + lb + wb;
    if (need > X.sc_bytes) {
        if (X.sc_buf && hipFree(X.sc_buf) != hipSuccess) return MPDP_EDEVICE;
        X.sc_buf = nullptr;
        X.sc_bytes = 0;
        if (hipMalloc(&X.sc_buf, need) != hipSuccess || !X.sc_buf) {
            (void)hipGetLastError();
            X.sc_buf = nullptr;
            return MPDP_ENOMEM;
        }
        X.sc_bytes = need;
    }
    char *b = static_cast<char *>(X.sc_buf);
    if (hipMemcpyAsync(b, feat.data(), 2 * feat.size(), hipMemcpyHostToDevice, X.s) != hipSuccess) return MPDP_EDEVICE;
    mpdp_status st = mpdp_scorer_forward(X.scorer, reinterpret_cast<const uint16_t *>(b), rows,
                                         reinterpret_cast<float *>(b + xb), b + xb + lb, wb, X.s);
    if (st != MPDP_OK) return st;
    if (hipMemcpyAsync(logit.data(), b + xb, 4 * (size_t)rows, hipMemcpyDeviceToHost, X.s) != hipSuccess)
        return MPDP_EDEVICE;
    if (hipStreamSynchronize(X.s) != hipSuccess) return MPDP_EDEVICE;
    return MPDP_OK;
}

// ---------------------------------------------------------------- UnionDP

// The learned partition phase over `units` (sorted by lowest relation):
// parts start as single units; each pass scores every union of two adjacent
// parts with at most k units together (part pairs ascending, parts numbered
// by their lowest unit) and joins the best-scored candidate (ties by pair
// order) if its score is positive; passes repeat until none joins.  `have` is false when
// the first pass joins nothing (the paper's order is used then).
mpdp_status learned_partition(ExactCtx &X, const std::vector<Unit> &units, const std::vector<int> &where, uint32_t k,
                              std::vector<std::vector<const Unit *>> &groups, bool &have) {
    const Graph &G = *X.G;
    std::vector<std::pair<uint32_t, uint32_t>> ue;
    for (size_t e = 0; e < G.eu.size(); ++e) {
        const int a = where[G.eu[e]], b = where[G.ev[e]];
        if (a != b) ue.push_back({(uint32_t)std::min(a, b), (uint32_t)std::max(a, b)});
    }
    std::sort(ue.begin(), ue.end());
    ue.erase(std::unique(ue.begin(), ue.end()), ue.end());
    std::vector<std::vector<uint32_t>> parts(units.size());
    std::vector<uint32_t> owner(units.size());
    for (uint32_t i = 0; i < units.size(); ++i) { parts[i] = {i}; owner[i] = i; }
    bool joined = false;
    std::vector<Bits> rels;
    std::vector<uint16_t> feat;
    std::vector<float> score;
    for (;;) {
        if (X.over_budget()) return MPDP_ETIMEOUT;
        std::vector<std::pair<uint32_t, uint32_t>> pairs;
        for (const auto &e : ue) {
            const uint32_t a = owner[e.first], b = owner[e.second];
            if (a != b && parts[a].size() + parts[b].size() <= k) pairs.push_back({std::min(a, b), std::max(a, b)});
        }
        std::sort(pairs.begin(), pairs.end());
        pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
        if (pairs.empty()) break;
        part_features(G, *X.P, units, parts, pairs, rels, feat);
        std::vector<float> label;
        if (X.plan_sets) {
            for (const auto &pr : pairs) {
                const Bits S = rels[pr.first] | rels[pr.second];
                label.push_back(X.plan_sets->count((uint32_t)S.w[0]) ? 1.f : 0.f);
            }
        }
        if (X.ex_x) {
            X.ex_x->insert(X.ex_x->end(), feat.begin(), feat.end());
            X.ex_y->insert(X.ex_y->end(), label.begin(), label.end());
        }
        if (X.teacher) {
            score.resize(pairs.size());
            for (size_t e = 0; e < pairs.size(); ++e) score[e] = label[e] * 2.f - 1.f;
        } else {
            const double t0 = now_ms();
            mpdp_status st = score_rows(X, feat, score);
            if (st != MPDP_OK) return st;
            X.st.ms_exact += now_ms() - t0;
        }
        std::vector<uint32_t> order(pairs.size());
        for (size_t e = 0; e < pairs.size(); ++e) order[e] = (uint32_t)e;
        std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
            return score[x] != score[y] ? score[x] > score[y] : x < y;
        });
        std::vector<char> touched(parts.size(), 0);
        bool did = false;
        for (uint32_t e : order) {
            if (!(score[e] > 0.f)) break;
            const uint32_t a = pairs[e].first, b = pairs[e].second;
            if (touched[a] || touched[b]) continue;
            parts[a].insert(parts[a].end(), parts[b].begin(), parts[b].end());
            parts[b].clear();
            touched[a] = touched[b] = 1;
            did = true;
            if (kOnePerPass) break;
        }
        if (!did) break;
        joined = true;
        std::vector<std::vector<uint32_t>> live;
        for (auto &p : parts)
            if (!p.empty()) { std::sort(p.begin(), p.end()); live.push_back(std::move(p)); }
        std::sort(live.begin(), live.end(), [](const std::vector<uint32_t> &x, const std::vector<uint32_t> &y) {
            return x[0] < y[0];
        });
        parts = std::move(live);
        for (uint32_t pi = 0; pi < parts.size(); ++pi)
            for (uint32_t u : parts[pi]) owner[u] = pi;
    }
    have = joined;
    groups.clear();
    if (!joined) return MPDP_OK;
    for (const auto &p : parts) {
        std::vector<const Unit *> g;
        for (uint32_t u : p) g.push_back(&units[u]);
        groups.push_back(std::move(g));
    }
    return MPDP_OK;
}

mpdp_status uniondp(ExactCtx &X, uint32_t k, int &result) {
    const Graph &G = *X.G;
    std::vector<Unit> units;
    for (uint32_t v = 0; v < G.n; ++v) units.push_back(Unit{G.single(v), X.P->leaf(v), v});
    std::vector<int> where(G.n, -1);
    // out of time: the current units joined greedily
    auto finish = [&]() {
        result = goo_units(G, *X.P, units);
        return result < 0 ? MPDP_ENOTCONNECTED : MPDP_ETIMEOUT;
    };
    while (units.size() > k) {
        if (X.over_budget()) return finish();
        X.st.rounds += 1;
        std::sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.low < b.low; });
        for (size_t i = 0; i < units.size(); ++i) units[i].rels.each([&](uint32_t v) { where[v] = (int)i; });
        std::vector<std::vector<const Unit *>> gl;
        bool have = false;
        if (X.scorer || X.teacher) {
            mpdp_status ls = learned_partition(X, units, where, k, gl, have);
            if (ls == MPDP_ETIMEOUT) return finish();
            if (ls != MPDP_OK) return ls;
        }
        if (!have) {  // the paper's partition phase
            std::vector<std::pair<uint32_t, uint32_t>> ue;
            for (size_t e = 0; e < G.eu.size(); ++e) {
                const int a = where[G.eu[e]], b = where[G.ev[e]];
                if (a != b) ue.push_back({(uint32_t)std::min(a, b), (uint32_t)std::max(a, b)});
            }
            std::sort(ue.begin(), ue.end());
            ue.erase(std::unique(ue.begin(), ue.end()), ue.end());
            std::vector<double> weight(ue.size());
            for (size_t e = 0; e < ue.size(); ++e)
                weight[e] = G.card_of(units[ue[e].first].rels | units[ue[e].second].rels);
            std::vector<uint32_t> parent(units.size()), size(units.size(), 1);
            for (size_t i = 0; i < units.size(); ++i) parent[i] = (uint32_t)i;
            auto find = [&](uint32_t x) {
                while (parent[x] != x) {
                    parent[x] = parent[parent[x]];
                    x = parent[x];
                }
                return x;
            };
            // edges by (size of both parts, weight, edge order), re-keyed as parts grow
            using Item = std::tuple<uint32_t, double, uint32_t>;
            std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
            for (size_t e = 0; e < ue.size(); ++e) heap.push(Item{2u, weight[e], (uint32_t)e});
            while (!heap.empty()) {
                const auto [sz, w, e] = heap.top();
                heap.pop();
                const uint32_t ri = find(ue[e].first), rj = find(ue[e].second);
                if (ri == rj) continue;
                const uint32_t cur = size[ri] + size[rj];
                if (cur > k) continue;  // sizes only grow
                if (cur != sz) {        // re-keyed: the parts have grown
                    heap.push(Item{cur, w, e});
                    continue;
                }
                const uint32_t lo = std::min(ri, rj), hi = std::max(ri, rj);
                parent[hi] = lo;
                size[lo] += size[hi];
            }
            std::map<uint32_t, std::vector<const Unit *>> groups;
            for (size_t i = 0; i < units.size(); ++i) groups[find((uint32_t)i)].push_back(&units[i]);
            for (auto &kv : groups) gl.push_back(kv.second);
        }
        std::vector<int> plans;
        mpdp_status s = exact_groups(X, gl, plans);
        if (s != MPDP_OK) return s;
        std::vector<Unit> next;
        for (size_t g = 0; g < gl.size(); ++g) {
            Bits r = gl[g][0]->rels;
            uint32_t low = gl[g][0]->low;
            for (size_t i = 1; i < gl[g].size(); ++i) {
                r = r | gl[g][i]->rels;
                low = std::min(low, gl[g][i]->low);
            }
            next.push_back(Unit{std::move(r), plans[g], low});
        }
        units = std::move(next);
    }
    if (X.over_budget()) return finish();
    std::vector<const Unit *> all;
    for (const Unit &u : units) all.push_back(&u);
    std::vector<int> plans;
    mpdp_status s = exact_groups(X, {all}, plans);
    if (s != MPDP_OK) return s;
    result = plans[0];
    return MPDP_OK;
}

// ---------------------------------------------------------------- validation and output

mpdp_status validate_large(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *card, const double *sel,
                           mpdp_cost_model cm, Graph &G) {
    if (n == 0) return MPDP_EINVAL;
    if (n > kLargeMaxRel) return MPDP_ETOOLARGE;
    if (cm != MPDP_COST_COUT && cm != MPDP_COST_PGLIKE) return MPDP_EINVAL;
    if (!card || (m > 0 && (!edges || !sel))) return MPDP_EINVAL;
    if ((uint64_t)m > (uint64_t)n * (n - 1) / 2) return MPDP_EINVAL;
    G.n = n;
    G.words = (n + 63) / 64;
    G.cm = cm;
    G.card.assign(card, card + n);
    for (uint32_t v = 0; v < n; ++v)
        if (!std::isfinite(card[v]) || !(card[v] >= 1.0)) return MPDP_EINVAL;
    G.lower.assign(n, {});
    G.adj.assign(n, {});
    std::unordered_set<uint64_t> seen;
    for (uint32_t i = 0; i < m; ++i) {
        const uint32_t u = edges[i].u, v = edges[i].v;
        if (u >= n || v >= n || u == v) return MPDP_EINVAL;
        if (!std::isfinite(sel[i]) || !(sel[i] > 0.0) || !(sel[i] <= 1.0)) return MPDP_EINVAL;
        const uint32_t a = std::min(u, v), b = std::max(u, v);
        if (!seen.insert(((uint64_t)a << 32) | b).second) return MPDP_EINVAL;
        G.eu.push_back(u);
        G.ev.push_back(v);
        G.sel.push_back(sel[i]);
        G.lower[b].push_back({a, sel[i]});
        G.adj[u].push_back(v);
        G.adj[v].push_back(u);
    }
    for (auto &l : G.lower) std::sort(l.begin(), l.end());
    std::vector<char> vis(n, 0);
    std::vector<uint32_t> stack{0};
    vis[0] = 1;
    uint32_t reached = 1;
    while (!stack.empty()) {
        const uint32_t v = stack.back();
        stack.pop_back();
        for (uint32_t u : G.adj[v])
            if (!vis[u]) { vis[u] = 1; ++reached; stack.push_back(u); }
    }
    return reached == n ? MPDP_OK : MPDP_ENOTCONNECTED;
}

void write_plan(Pool &P, int root, mpdp_large_node *out, uint32_t n) {
    const Graph &G = *P.G;
    for (uint32_t v = 0; v < n; ++v)
        out[v] = mpdp_large_node{-1, -1, v, 1u, MPDP_OP_SCAN, 0u, G.scan_cost(v), G.card[v]};
    uint32_t next = n;
    // post-order, left child first
    std::vector<std::pair<int, int>> st{{root, 0}};
    std::vector<int> idx;  // results of finished children
    while (!st.empty()) {
        auto &[x, stage] = st.back();
        const PNode &p = P.nodes[x];
        if (p.leaf >= 0) {
            idx.push_back(p.leaf);
            st.pop_back();
            continue;
        }
        if (stage == 0) { stage = 1; st.push_back({p.l, 0}); continue; }
        if (stage == 1) { stage = 2; st.push_back({p.r, 0}); continue; }
        const int ri = idx.back(); idx.pop_back();
        const int li = idx.back(); idx.pop_back();
        out[next] = mpdp_large_node{li, ri, p.rels.lowest(), p.rels.count(), p.op, 0u, p.cost, p.card};
        idx.push_back((int)next);
        ++next;
        st.pop_back();
    }
}

}  // namespace

extern "C" mpdp_status mpdp_optimize_large_budget(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                                  const double *cardinalities, const double *selectivities,
                                                  mpdp_cost_model cost_model, mpdp_large_method method, uint32_t k,
                                                  const void *d_scorer, double budget_ms, void *hip_stream,
                                                  mpdp_large_node *plan_out, double *cost_out,
                                                  mpdp_large_stats *stats_out) {
    const double t0 = now_ms();
    if (!plan_out || !cost_out) return MPDP_EINVAL;
    if (!std::isfinite(budget_ms) || budget_ms < 0.0) return MPDP_EINVAL;
    if (method != MPDP_LARGE_GOO && method != MPDP_LARGE_IDP2 && method != MPDP_LARGE_UNIONDP &&
        method != MPDP_LARGE_UNIONDP_LEARNED)
        return MPDP_EINVAL;
    if (method == MPDP_LARGE_UNIONDP_LEARNED && !d_scorer) return MPDP_EINVAL;
    if (method != MPDP_LARGE_GOO && (k < 2 || k > kLargeMaxK)) return MPDP_EINVAL;
    Graph G;
    mpdp_status st = validate_large(n, m, edges, cardinalities, selectivities, cost_model, G);
    if (st != MPDP_OK) return st;
    Pool P;
    P.G = &G;
    P.leaf_of.assign(n, -1);
    P.nodes.reserve(8 * (size_t)n);
    ExactCtx X;
    X.G = &G;
    X.P = &P;
    X.s = static_cast<hipStream_t>(hip_stream);
    X.where.assign(n, -1);
    X.t0 = t0;
    X.budget_ms = method == MPDP_LARGE_GOO ? 0.0 : budget_ms;
    if (method == MPDP_LARGE_UNIONDP_LEARNED) X.scorer = d_scorer;
    int root = -1;
    if (method == MPDP_LARGE_UNIONDP || method == MPDP_LARGE_UNIONDP_LEARNED) {
        st = uniondp(X, k, root);
    } else {
        root = goo(G, P);
        if (root < 0) return MPDP_ENOTCONNECTED;
        if (method == MPDP_LARGE_IDP2) {
            const int start = root;
            st = idp2(X, start, k, root);
        }
    }
    if (st != MPDP_OK && st != MPDP_ETIMEOUT) return st;
    P.recost(root);
    write_plan(P, root, plan_out, n);
    *cost_out = P.nodes[root].cost;
    if (stats_out) {
        X.st.ms_total = now_ms() - t0;
        *stats_out = X.st;
    }
    return st;
}

extern "C" mpdp_status mpdp_optimize_large(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                           const double *cardinalities, const double *selectivities,
                                           mpdp_cost_model cost_model, mpdp_large_method method, uint32_t k,
                                           const void *d_scorer, void *hip_stream, mpdp_large_node *plan_out,
                                           double *cost_out, mpdp_large_stats *stats_out) {
    return mpdp_optimize_large_budget(n, m, edges, cardinalities, selectivities, cost_model, method, k, d_scorer,
                                      0.0, hip_stream, plan_out, cost_out, stats_out);
}

extern "C" mpdp_status mpdp_large_examples(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *cardinalities,
                                          const double *selectivities, mpdp_cost_model cost_model, uint32_t k,
                                          const void *d_scorer, const uint32_t *plan_sets, uint32_t nsets,
                                          void *hip_stream, uint16_t *features_out, float *labels_out,
                                          uint32_t max_examples, uint32_t *count_out) {
    if (!plan_sets || !count_out || (max_examples > 0 && (!features_out || !labels_out))) return MPDP_EINVAL;
    if (n > 32) return MPDP_ETOOLARGE;
    if (k < 2 || k > kLargeMaxK) return MPDP_EINVAL;
    Graph G;
    mpdp_status st = validate_large(n, m, edges, cardinalities, selectivities, cost_model, G);
    if (st != MPDP_OK) return st;
    std::unordered_set<uint32_t> sets(plan_sets, plan_sets + nsets);
    std::vector<uint16_t> ex;
    std::vector<float> ey;
    Pool P;
    P.G = &G;
    P.leaf_of.assign(n, -1);
    ExactCtx X;
    X.G = &G;
    X.P = &P;
    X.s = static_cast<hipStream_t>(hip_stream);
    X.where.assign(n, -1);
    X.scorer = d_scorer;
    X.teacher = d_scorer == nullptr;
    X.plan_sets = &sets;
    X.ex_x = &ex;
    X.ex_y = &ey;
    int root = -1;
    st = uniondp(X, k, root);
    if (st != MPDP_OK) return st;
    const uint32_t count = (uint32_t)ey.size();
    *count_out = count;
    if (count > max_examples) return MPDP_ENOMEM;
    std::memcpy(features_out, ex.data(), 2 * ex.size());
    std::memcpy(labels_out, ey.data(), 4 * ey.size());
    return MPDP_OK;
}
