/*
 * CPU oracle for the MPDP join-order dynamic program.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or constant with the HIP implementation; the two only agree on the
 * written definitions below.
 *
 * Built with gcc -O2 -ffp-contract=off (no fast-math): every floating-point
 * expression is evaluated exactly as written, left to right.
 *
 * Definitions (readings of the paper, each stated once here):
 *
 *  card(S)  The paper never specifies cardinality estimation (Section 7.1,
 *           cost model paragraph).  card(S) is a function of S alone:
 *             c = 1.0
 *             for v in S ascending:
 *                 c = c * card[v]
 *                 for u in S, u < v, (u,v) an edge, ascending: c = c * sel(u,v)
 *             card(S) = (c < 1.0) ? 1.0 : c
 *
 *  C_out    (Section 7.1, after Neumann 2018) cost({v}) = 0,
 *           cost(L join R) = (cost(L) + cost(R)) + card(L u R).
 *
 *  PG-like  The paper's PostgreSQL-like model has no published formulas
 *           (Section 7.1).  Our own, from PostgreSQL's default constants
 *           cpu_tuple_cost = 0.01 and cpu_operator_cost = 0.0025:
 *             cost({v}) = 0.01 * card[v]
 *             HJ(L,R) = (((cL + cR) + 0.0125 * card(R)) + 0.0025 * card(L)) + 0.01 * card(S)
 *             NL(L,R) = ((cL + cR) + (0.0025 * card(L)) * card(R)) + 0.01 * card(S)
 *           a join takes HJ if HJ <= NL, else NL.
 *
 *  Best plan  The paper keeps the first strictly cheaper plan in enumeration
 *           order (Alg. 1), which is order dependent.  Here every candidate
 *           (L, R, op) is ranked by the key (cost, L as an unsigned bitmap,
 *           op with HASH < NESTLOOP) and the smallest key wins, so the memo
 *           does not depend on enumeration order.
 *
 *  Counters  evaluated: candidate join pairs the algorithm looks at.
 *           ccp_ordered: candidates that pass the CCP block, counting (L,R)
 *           and (R,L) separately (Section 2.1: "including the symmetric ones").
 *
 * Memo layout used by every routine here: dense arrays indexed by the set
 * bitmap S (size 2^n): cost[S], card[S], left[S], op[S]; left[S] == 0 marks a
 * set without a plan (not connected, or not reached).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OP_SCAN 0
#define OP_HASH 1
#define OP_NESTLOOP 2
#define OP_JOIN 3

#define CM_COUT 0
#define CM_PGLIKE 1

typedef struct {
    int n;
    int cost_model;
    uint32_t adj[32];
    double card[32];
    double sel[32][32];
    int has_bcost;      /* relations are intermediate results with given plan costs */
    double bcost[32];
} og;

typedef struct {
    double *cost;
    double *card;
    uint32_t *left;
    uint8_t *op;
} omemo;

typedef struct {
    uint64_t evaluated;
    uint64_t ccp_ordered;
    uint64_t connected_sets; /* |S| >= 2 */
} ocount;

/* ---------- input ---------- */

static int og_build(og *g, int n, int m, const uint32_t *edges, const double *card,
                    const double *sel, int cost_model)
{
    if (n < 1 || n > 32) return -1;
    memset(g, 0, sizeof(*g));
    g->n = n;
    g->cost_model = cost_model;
    for (int v = 0; v < n; v++) g->card[v] = card[v];
    for (int i = 0; i < m; i++) {
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= (uint32_t)n || v >= (uint32_t)n || u == v) return -1;
        g->adj[u] |= 1u << v;
        g->adj[v] |= 1u << u;
        g->sel[u][v] = sel[i];
        g->sel[v][u] = sel[i];
    }
    return 0;
}

static inline uint32_t bit(int v) { return 1u << v; }
static inline int lowest(uint32_t S) { return __builtin_ctz(S); }
static inline uint32_t below(int v) { return v >= 32 ? 0xffffffffu : (bit(v) - 1u); }

/* ---------- grow / connected (Section 3.2.1) ---------- */

/* All vertices of `restriction` reachable from `source` inside `restriction`. */
static uint32_t grow(const og *g, uint32_t source, uint32_t restriction)
{
    uint32_t visited = 0, frontier = source;
    while (frontier) {
        int x = lowest(frontier);
        visited |= bit(x);
        frontier = (frontier | (g->adj[x] & restriction)) & ~visited;
    }
    return visited;
}

/* G[S] connected: grow from the lowest vertex of S reaches all of S. */
static int connected(const og *g, uint32_t S)
{
    if (!S) return 0;
    return grow(g, bit(lowest(S)), S) == S;
}

/* An edge joins a vertex of A with a vertex of B. */
static int adjacent(const og *g, uint32_t A, uint32_t B)
{
    for (uint32_t T = A; T; T &= T - 1)
        if (g->adj[lowest(T)] & B) return 1;
    return 0;
}

/* ---------- cardinality and cost ---------- */

static double card_of(const og *g, uint32_t S)
{
    double c = 1.0;
    for (int v = 0; v < g->n; v++) {
        if (!(S & bit(v))) continue;
        c = c * g->card[v];
        for (int u = 0; u < v; u++)
            if ((S & bit(u)) && (g->adj[v] & bit(u))) c = c * g->sel[u][v];
    }
    return (c < 1.0) ? 1.0 : c;
}

/* Cost of the plan of a single relation: a scan (0 under C_out, one tuple
 * cost per row under the PostgreSQL-like model), or, for a relation that
 * stands for an already planned intermediate result, that plan's cost. */
static double base_cost(const og *g, int v)
{
    if (g->has_bcost) return g->bcost[v];
    return g->cost_model == CM_PGLIKE ? 0.01 * g->card[v] : 0.0;
}

/* Cost of joining memoised plans of L (outer/left) and R (inner/right). */
static void join_cost(const og *g, const omemo *M, uint32_t L, uint32_t R, double cardS,
                      double *cost, uint8_t *op)
{
    double cL = M->cost[L], cR = M->cost[R];
    if (g->cost_model == CM_COUT) {
        *cost = (cL + cR) + cardS;
        *op = OP_JOIN;
        return;
    }
    double kL = M->card[L], kR = M->card[R];
    double hj = (((cL + cR) + 0.0125 * kR) + 0.0025 * kL) + 0.01 * cardS;
    double nl = ((cL + cR) + (0.0025 * kL) * kR) + 0.01 * cardS;
    if (hj <= nl) { *cost = hj; *op = OP_HASH; }
    else { *cost = nl; *op = OP_NESTLOOP; }
}

/* Key order: cost, then left bitmap, then op. */
static int key_less(double c1, uint32_t l1, uint8_t o1, double c2, uint32_t l2, uint8_t o2)
{
    if (c1 != c2) return c1 < c2;
    if (l1 != l2) return l1 < l2;
    return o1 < o2;
}

/* Best plan of S so far, held while S is being evaluated. */
typedef struct { double cost; uint32_t left; uint8_t op; int have; } best_t;

static void consider(const og *g, const omemo *M, uint32_t L, uint32_t R, double cardS, best_t *b)
{
    double c; uint8_t op;
    join_cost(g, M, L, R, cardS, &c, &op);
    if (!b->have || key_less(c, L, op, b->cost, b->left, b->op)) {
        b->cost = c; b->left = L; b->op = op; b->have = 1;
    }
}

static void memo_init(const og *g, omemo *M)
{
    size_t N = (size_t)1 << g->n;
    for (size_t s = 0; s < N; s++) { M->left[s] = 0; M->op[s] = 0; M->cost[s] = INFINITY; M->card[s] = 0.0; }
    for (int v = 0; v < g->n; v++) {
        M->cost[bit(v)] = base_cost(g, v);
        M->card[bit(v)] = g->card[v];
        M->op[bit(v)] = OP_SCAN;
    }
}

static void memo_store(omemo *M, uint32_t S, const best_t *b, double cardS)
{
    M->cost[S] = b->cost; M->card[S] = cardS; M->left[S] = b->left; M->op[S] = b->op;
}

/* Next bitmap with the same popcount (used to walk all i-subsets of n). */
static uint32_t next_same_popcount(uint32_t x)
{
    uint32_t c = x & -x, r = x + c;
    return (((r ^ x) >> 2) / c) | r;
}

/* ---------- DPSUB (Alg. 1, Section 2.2) ---------- */

int oracle_dpsub(int n, int m, const uint32_t *edges, const double *card, const double *sel,
                 int cost_model, double *mcost, double *mcard, uint32_t *mleft, uint8_t *mop,
                 uint64_t *counters)
{
    og g;
    if (n > 20 || og_build(&g, n, m, edges, card, sel, cost_model)) return -1;
    omemo M = {mcost, mcard, mleft, mop};
    ocount C = {0, 0, 0};
    memo_init(&g, &M);
    for (int i = 2; i <= n; i++) {
        /* S_i: connected subsets of size i */
        uint32_t last = (n == 32) ? 0 : bit(n);
        for (uint32_t S = below(i); S < last && S != 0; S = next_same_popcount(S)) {
            if (!connected(&g, S)) continue;
            C.connected_sets++;
            double cardS = card_of(&g, S);
            best_t b = {0, 0, 0, 0};
            /* all S_left subset of S, empty and full included */
            uint32_t sub = 0;
            do {
                C.evaluated++;
                uint32_t L = sub, R = S & ~sub;
                int ok = 1;
                if (R == 0 || L == 0) ok = 0;                 /* CCP block begins */
                else if (!connected(&g, L)) ok = 0;
                else if (!connected(&g, R)) ok = 0;
                else if ((R & L) != 0) ok = 0;
                else if (!adjacent(&g, L, R)) ok = 0;          /* CCP block ends */
                if (ok) {
                    C.ccp_ordered++;
                    consider(&g, &M, L, R, cardS, &b);
                }
                sub = (sub - S) & S; /* next subset of S in increasing order */
            } while (sub != 0);
            memo_store(&M, S, &b, cardS);
        }
    }
    counters[0] = C.evaluated; counters[1] = C.ccp_ordered; counters[2] = C.connected_sets;
    return 0;
}

/* ---------- Find-Blocks: Hopcroft-Tarjan on G[S] (Section 3.2.2) ---------- */

typedef struct {
    const og *g;
    uint32_t S;
    int disc[32], low[32], timer;
    int eu[512], ev[512], esp;
    uint32_t blocks[32];
    int nb;
} htstate;

static void ht_dfs(htstate *h, int u, int parent)
{
    h->disc[u] = h->low[u] = ++h->timer;
    uint32_t nbrs = h->g->adj[u] & h->S;
    for (uint32_t T = nbrs; T; T &= T - 1) {
        int v = lowest(T);
        if (!h->disc[v]) {
            h->eu[h->esp] = u; h->ev[h->esp] = v; h->esp++;
            ht_dfs(h, v, u);
            if (h->low[v] < h->low[u]) h->low[u] = h->low[v];
            if (h->low[v] >= h->disc[u]) {
                /* u separates: pop the edges of one block */
                uint32_t blk = 0;
                for (;;) {
                    h->esp--;
                    int a = h->eu[h->esp], b = h->ev[h->esp];
                    blk |= bit(a) | bit(b);
                    if (a == u && b == v) break;
                }
                h->blocks[h->nb++] = blk;
            }
        } else if (v != parent && h->disc[v] < h->disc[u]) {
            h->eu[h->esp] = u; h->ev[h->esp] = v; h->esp++;
            if (h->disc[v] < h->low[u]) h->low[u] = h->disc[v];
        }
    }
}

/* Blocks (biconnected components) of G[S] for a connected S with |S| >= 2. */
static int find_blocks(const og *g, uint32_t S, uint32_t *out)
{
    htstate h;
    memset(&h, 0, sizeof(h));
    h.g = g; h.S = S;
    ht_dfs(&h, lowest(S), -1);
    for (int i = 0; i < h.nb; i++) out[i] = h.blocks[i];
    return h.nb;
}

int oracle_blocks(int n, int m, const uint32_t *edges, uint32_t S, uint32_t *out)
{
    og g;
    double card[32], sel[1024];
    for (int i = 0; i < 32; i++) card[i] = 1.0;
    for (int i = 0; i < m && i < 1024; i++) sel[i] = 1.0;
    if (m > 1024 || og_build(&g, n, m, edges, card, sel, CM_COUT)) return -1;
    if (__builtin_popcount(S) < 2 || !connected(&g, S)) return 0;
    return find_blocks(&g, S, out);
}

/* ---------- MPDP (Alg. 2 on trees, Alg. 3 otherwise, Section 3) ---------- */

static int graph_is_tree(const og *g, int m)
{
    uint32_t all = (g->n == 32) ? 0xffffffffu : (bit(g->n) - 1u);
    return m == g->n - 1 && connected(g, all);
}

static int mpdp_run(og *gp, int m, int force_general, double *mcost, double *mcard, uint32_t *mleft,
                    uint8_t *mop, uint64_t *counters, int nthreads);

int oracle_mpdp(int n, int m, const uint32_t *edges, const double *card, const double *sel,
                int cost_model, int force_general, double *mcost, double *mcard, uint32_t *mleft,
                uint8_t *mop, uint64_t *counters)
{
    og g;
    if (n > 30 || og_build(&g, n, m, edges, card, sel, cost_model)) return -1;
    return mpdp_run(&g, m, force_general, mcost, mcard, mleft, mop, counters, 1);
}

/* oracle_mpdp with the sets of each level split over nthreads threads. */
int oracle_mpdp_threads(int n, int m, const uint32_t *edges, const double *card, const double *sel,
                        int cost_model, int force_general, int nthreads, double *mcost, double *mcard,
                        uint32_t *mleft, uint8_t *mop, uint64_t *counters)
{
    og g;
    if (n > 30 || og_build(&g, n, m, edges, card, sel, cost_model)) return -1;
    return mpdp_run(&g, m, force_general, mcost, mcard, mleft, mop, counters, nthreads);
}

/* MPDP where every relation carries the cost of its plan (bcost[v]): the
 * exact step of the large-query heuristics, whose relations may be
 * intermediate results planned earlier. */
int oracle_mpdp_bc(int n, int m, const uint32_t *edges, const double *card, const double *sel,
                   int cost_model, const double *bcost, double *mcost, double *mcard, uint32_t *mleft,
                   uint8_t *mop, uint64_t *counters)
{
    og g;
    if (n > 30 || og_build(&g, n, m, edges, card, sel, cost_model)) return -1;
    g.has_bcost = 1;
    for (int v = 0; v < n; v++) g.bcost[v] = bcost[v];
    return mpdp_run(&g, m, 0, mcost, mcard, mleft, mop, counters, 1);
}

/* Evaluate one set S of the current level: skip it if G[S] is not
 * connected, else find its best plan from memo entries of smaller sets. */
static void mpdp_set(const og *g, omemo *M, int tree, uint32_t S, ocount *C)
{
    if (!connected(g, S)) return;
    C->connected_sets++;
    double cardS = card_of(g, S);
    best_t b = {0, 0, 0, 0};
    if (tree) {
        /* Alg. 2: one join pair per edge of the tree G[S]; both
           orientations of each pair are costed. */
        for (uint32_t T = S; T; T &= T - 1) {
            int v = lowest(T);
            for (uint32_t U = g->adj[v] & S & below(v); U; U &= U - 1) {
                int u = lowest(U);
                uint32_t L = grow(g, bit(u), S & ~bit(v));
                uint32_t R = S & ~L;
                C->evaluated += 2;
                C->ccp_ordered += 2;
                consider(g, M, L, R, cardS, &b);
                consider(g, M, R, L, cardS, &b);
            }
        }
    } else {
        /* Alg. 3: vertex-based enumeration inside each block, then
           grow the block pair to a pair of S. */
        uint32_t blocks[32];
        int nb = find_blocks(g, S, blocks);
        for (int k = 0; k < nb; k++) {
            uint32_t blk = blocks[k];
            for (uint32_t lb = (0u - blk) & blk; lb != 0; lb = (lb - blk) & blk) {
                if (lb == blk) continue; /* proper, non-empty subsets only */
                C->evaluated++;
                uint32_t rb = blk & ~lb;
                if (rb == 0 || lb == 0) continue;
                if (!connected(g, lb)) continue;
                if (!connected(g, rb)) continue;
                if ((rb & lb) != 0) continue;
                if (!adjacent(g, lb, rb)) continue;
                C->ccp_ordered++;
                uint32_t L = grow(g, lb, S & ~rb);
                uint32_t R = S & ~L;
                consider(g, M, L, R, cardS, &b);
            }
        }
    }
    memo_store(M, S, &b, cardS);
}

/* Every i-subset of the n relations whose top `hi` relations (n - hi and
 * up) are exactly the pattern h: the low part walks the subsets of the
 * remaining relations with the remaining popcount. */
static void mpdp_part(const og *g, omemo *M, int tree, int i, int hi, uint32_t h, ocount *C)
{
    int n = g->n, lo = n - hi, want = i - __builtin_popcount(h);
    if (want < 0 || want > lo) return;
    uint32_t top = lo >= 32 ? 0u : h << lo;
    if (want == 0) { mpdp_set(g, M, tree, top, C); return; }
    uint64_t last = (uint64_t)1 << lo;
    for (uint64_t l = below(want); l < last; l = next_same_popcount((uint32_t)l)) {
        mpdp_set(g, M, tree, top | (uint32_t)l, C);
        if (l == ((uint64_t)below(want) << (lo - want))) break; /* the last i-subset of the low part */
    }
}

/* The level loop (Section 5, Alg. 5): sets of one size depend only on
 * smaller sets, so with nthreads > 1 the sets of a level are split by the
 * pattern of their top relations and evaluated in parallel.  The memo and
 * the counters are the same whatever nthreads is. */
static int mpdp_run(og *gp, int m, int force_general, double *mcost, double *mcard, uint32_t *mleft,
                    uint8_t *mop, uint64_t *counters, int nthreads)
{
    og g = *gp;
    int n = g.n;
    omemo M = {mcost, mcard, mleft, mop};
    ocount C = {0, 0, 0};
    memo_init(&g, &M);
    int tree = !force_general && graph_is_tree(&g, m);
    int hi = nthreads > 1 ? (n < 10 ? n : 10) : 0;
    for (int i = 2; i <= n; i++) {
        uint64_t ev = 0, cc = 0, cs = 0;
        int64_t parts = (int64_t)1 << hi;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 1 ? nthreads : 1) reduction(+ : ev, cc, cs)
        for (int64_t h = 0; h < parts; h++) {
            ocount P = {0, 0, 0};
            mpdp_part(&g, &M, tree, i, hi, (uint32_t)h, &P);
            ev += P.evaluated; cc += P.ccp_ordered; cs += P.connected_sets;
        }
        C.evaluated += ev; C.ccp_ordered += cc; C.connected_sets += cs;
    }
    counters[0] = C.evaluated; counters[1] = C.ccp_ordered; counters[2] = C.connected_sets;
    return 0;
}

/* ---------- DPccp csg-cmp enumeration (Moerkotte & Neumann, VLDB 2006) ----------
 * Each unordered csg-cmp pair is produced once.  Used to count pairs and,
 * with the pairs bucketed by |S1 u S2|, as a third DP that does not depend on
 * the emission order. */

typedef struct {
    const og *g;
    uint64_t count;
    uint64_t *per_level;  /* optional: pairs counted by |S1 u S2| */
    uint32_t *pairs;      /* optional: 2 words per pair, bucketed by level */
    uint64_t *cursor;     /* per-level write cursor into pairs */
} ccpenum;

static uint32_t neigh(const og *g, uint32_t S)
{
    uint32_t N = 0;
    for (uint32_t T = S; T; T &= T - 1) N |= g->adj[lowest(T)];
    return N & ~S;
}

static void emit_pair(ccpenum *e, uint32_t S1, uint32_t S2)
{
    int lvl = __builtin_popcount(S1 | S2);
    e->count++;
    if (e->per_level) e->per_level[lvl]++;
    if (e->pairs) {
        uint64_t at = e->cursor[lvl]++;
        e->pairs[2 * at] = S1;
        e->pairs[2 * at + 1] = S2;
    }
}

static void enum_cmp_rec(ccpenum *e, uint32_t S1, uint32_t S2, uint32_t X)
{
    uint32_t N = neigh(e->g, S2) & ~X;
    if (!N) return;
    for (uint32_t s = (0u - N) & N; s; s = (s - N) & N) emit_pair(e, S1, S2 | s);
    for (uint32_t s = (0u - N) & N; s; s = (s - N) & N) enum_cmp_rec(e, S1, S2 | s, X | N);
}

static void emit_csg(ccpenum *e, uint32_t S1)
{
    int mn = lowest(S1);
    uint32_t X = S1 | below(mn + 1);
    uint32_t N = neigh(e->g, S1) & ~X;
    for (int v = 31; v >= 0; v--) {
        if (!(N & bit(v))) continue;
        emit_pair(e, S1, bit(v));
        enum_cmp_rec(e, S1, bit(v), X | (below(v + 1) & N));
    }
}

static void enum_csg_rec(ccpenum *e, uint32_t S, uint32_t X)
{
    uint32_t N = neigh(e->g, S) & ~X;
    if (!N) return;
    for (uint32_t s = (0u - N) & N; s; s = (s - N) & N) emit_csg(e, S | s);
    for (uint32_t s = (0u - N) & N; s; s = (s - N) & N) enum_csg_rec(e, S | s, X | N);
}

static void dpccp_enumerate(ccpenum *e)
{
    for (int v = e->g->n - 1; v >= 0; v--) {
        emit_csg(e, bit(v));
        enum_csg_rec(e, bit(v), below(v + 1));
    }
}

uint64_t oracle_count_ccp(int n, int m, const uint32_t *edges)
{
    og g;
    double card[32], *sel = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    for (int i = 0; i < 32; i++) card[i] = 1.0;
    for (int i = 0; i < m; i++) sel[i] = 1.0;
    int bad = og_build(&g, n, m, edges, card, sel, CM_COUT);
    free(sel);
    if (bad) return 0;
    ccpenum e;
    memset(&e, 0, sizeof(e));
    e.g = &g;
    dpccp_enumerate(&e);
    return e.count;
}

int oracle_dpccp(int n, int m, const uint32_t *edges, const double *card, const double *sel,
                 int cost_model, double *mcost, double *mcard, uint32_t *mleft, uint8_t *mop,
                 uint64_t *counters)
{
    og g;
    if (n > 26 || og_build(&g, n, m, edges, card, sel, cost_model)) return -1;
    uint64_t per_level[34], cursor[34];
    memset(per_level, 0, sizeof(per_level));
    ccpenum e;
    memset(&e, 0, sizeof(e));
    e.g = &g;
    e.per_level = per_level;
    dpccp_enumerate(&e);                     /* pass 1: count per level */
    uint64_t total = e.count, off = 0;
    for (int i = 0; i < 34; i++) { cursor[i] = off; off += per_level[i]; }
    uint32_t *pairs = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (total ? total : 1));
    if (!pairs) return -2;
    memset(&e, 0, sizeof(e));
    e.g = &g;
    e.pairs = pairs;
    e.cursor = cursor;
    dpccp_enumerate(&e);                     /* pass 2: store, bucketed by level */
    omemo M = {mcost, mcard, mleft, mop};
    memo_init(&g, &M);
    uint64_t connected_sets = 0, p = 0;
    for (int i = 0; i < 34; i++) {           /* DP in level order */
        for (uint64_t end = p + per_level[i]; p < end; p++) {
            uint32_t S1 = pairs[2 * p], S2 = pairs[2 * p + 1], S = S1 | S2;
            double cardS = card_of(&g, S);
            best_t b;
            b.have = M.left[S] != 0;
            b.cost = M.cost[S]; b.left = M.left[S]; b.op = M.op[S];
            if (!b.have) connected_sets++;
            consider(&g, &M, S1, S2, cardS, &b);
            consider(&g, &M, S2, S1, cardS, &b);
            memo_store(&M, S, &b, cardS);
        }
    }
    free(pairs);
    counters[0] = 2 * total; counters[1] = 2 * total; counters[2] = connected_sets;
    return 0;
}

/* ---------- small exported helpers for the tests ---------- */

int oracle_card(int n, int m, const uint32_t *edges, const double *card, const double *sel,
                uint32_t S, double *out)
{
    og g;
    if (og_build(&g, n, m, edges, card, sel, CM_COUT)) return -1;
    *out = card_of(&g, S);
    return 0;
}

uint32_t oracle_grow(int n, int m, const uint32_t *edges, uint32_t source, uint32_t restriction)
{
    og g;
    double card[32], sel[1024];
    for (int i = 0; i < 32; i++) card[i] = 1.0;
    for (int i = 0; i < m && i < 1024; i++) sel[i] = 1.0;
    if (m > 1024 || og_build(&g, n, m, edges, card, sel, CM_COUT)) return 0;
    return grow(&g, source, restriction);
}

/* Alg. 3's candidate count for one S: sum over blocks of (2^b - 2). */
uint64_t oracle_mpdp_candidates(int n, int m, const uint32_t *edges, uint32_t S)
{
    uint32_t blocks[32];
    int nb = oracle_blocks(n, m, edges, S, blocks);
    uint64_t t = 0;
    for (int i = 0; i < nb; i++) t += (1ull << __builtin_popcount(blocks[i])) - 2;
    return t;
}
