"""CPU oracle of the large-query heuristics (Section 4): IDP2 with GOO as
its initial plan (Section 4.1), UnionDP (Section 4.2, Alg. 4), and GOO on
its own.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
benchmark's CPU-baseline leg may use it; the library never does.

Plain Python over bitsets held in Python integers (bit v = relation v), so
any number of relations works; the exact step is the oracle's MPDP
(``oracle.mpdp``), run on a query whose relations are "units": base
relations or intermediate results planned earlier.

Readings of the points the paper leaves open (listed in the design notes):

H1  card(S) of any relation set is the canonical product of the exact DP
    (relations ascending, card[v] then the selectivities of the edges to
    smaller members, ascending; clamped below at 1), whatever the size of S.
H2  A plan is scored by re-costing it over the base relations: every join
    node takes the cheaper orientation and operator under the cost model
    (key: cost, then the left side's relation set read as a binary number,
    then HASH before NESTLOOP), leaves cost their scan.  GOO, IDP2 and
    UnionDP plans are all reported this way.
H3  A unit is passed to the exact step as one relation: its card is card(H1)
    of its relation set, its base cost is its plan's cost (H2); two units
    are joined by one edge whose selectivity is the product of the base
    selectivities between them, in edge-list order, clamped below at the
    smallest normal double.  Units are labelled by their lowest relation,
    ascending.
H4  GOO joins, at every step, the two connected trees whose union has the
    smallest card(H1); ties go to the pair with the smallest lowest
    relations (smaller of the two first, then the larger).
H5  IDP2 picks, among the subtrees with 2..k units, the one with the highest
    cost (H2); ties go to the subtree whose lowest relation is smaller.  The
    picked units are re-planned by the exact step and become one unit.
H6  UnionDP: the size of a partition counts units; the weight of an edge
    between two units is card(H1) of their union, fixed for the level; edges
    are taken in increasing (current size of the two partitions together,
    weight, edge order), re-keyed as partitions grow, and join their
    partitions when that size is at most k.  Every partition of two or more
    units is planned by the exact step and becomes one unit; the graph of
    units is then processed again until it has at most k units, which the
    exact step plans as a whole.

The learned variant (not in the paper; the scorer of mpdp_scorer.h):
L1  features of a candidate union of two parts: part_features() below.
L2  the partition phase joins parts one at a time, the best-scored union
    first, re-scoring after every join: learned_partition() below.
L3  training label of a union: 1 iff its relation set is a node of the
    optimal plan (the exact DP's, on queries small enough for it).
L4  a round in which the learned phase joins nothing uses the paper's order.
"""
from __future__ import annotations

import heapq
import math
import sys
from dataclasses import dataclass

import numpy as np

import oracle

COUT, PGLIKE = oracle.COST_COUT, oracle.COST_PGLIKE
OP_SCAN, OP_HASH, OP_NESTLOOP, OP_JOIN = oracle.OP_SCAN, oracle.OP_HASH, oracle.OP_NESTLOOP, 3
DBL_MIN = float(np.finfo(np.float64).tiny)

# plans are walked recursively; a plan is at most n joins deep
sys.setrecursionlimit(max(sys.getrecursionlimit(), 20000))


class Graph:
    """Base query data with lower-neighbour lists for the canonical product."""

    def __init__(self, q):
        self.q = q
        self.n = q.n
        self.card = [float(x) for x in q.card]
        self.edges = [(int(u), int(v)) for u, v in q.edges.tolist()]
        self.sel = [float(x) for x in q.sel]
        self.lower = [[] for _ in range(self.n)]  # (u, sel) for edges (u, v), u < v, u ascending
        for (a, b), s in zip(self.edges, self.sel):
            u, v = min(a, b), max(a, b)
            self.lower[v].append((u, s))
        for v in range(self.n):
            self.lower[v].sort()
        self.adj = [0] * self.n
        for a, b in self.edges:
            self.adj[a] |= 1 << b
            self.adj[b] |= 1 << a

    def card_of(self, S: int) -> float:
        """H1: canonical product over S, clamped below at 1."""
        c = 1.0
        v = 0
        T = S
        while T:
            if T & 1:
                c = c * self.card[v]
                for u, s in self.lower[v]:
                    if S >> u & 1:
                        c = c * s
            T >>= 1
            v += 1
        return 1.0 if c < 1.0 else c

    def scan_cost(self, v: int, cm: int) -> float:
        return 0.01 * self.card[v] if cm == PGLIKE else 0.0


def lowest(S: int) -> int:
    return (S & -S).bit_length() - 1


# ------------------------------------------------------------------ plans
#
# A plan is a nested tuple: ("leaf", v) or ("join", A, B) with A, B plans.
# Re-costing (H2) returns a Node tree with cost, card, orientation and op.

@dataclass
class Node:
    rels: int
    cost: float
    card: float
    op: int
    left: "Node | None" = None
    right: "Node | None" = None


def recost(G: Graph, plan, cm: int, cache=None) -> Node:
    """H2 over the base relations (bottom-up)."""
    if plan[0] == "leaf":
        v = plan[1]
        return Node(1 << v, G.scan_cost(v, cm), G.card[v], OP_SCAN)
    a = recost(G, plan[1], cm, cache)
    b = recost(G, plan[2], cm, cache)
    S = a.rels | b.rels
    if cache is not None and S in cache:
        cS = cache[S]
    else:
        cS = G.card_of(S)
        if cache is not None:
            cache[S] = cS
    base = a.cost + b.cost
    if cm == COUT:
        l, r = (a, b) if a.rels < b.rels else (b, a)
        return Node(S, base + cS, cS, OP_JOIN, l, r)
    out = 0.01 * cS
    cands = []
    for L, R in ((a, b), (b, a)):
        hj = ((base + 0.0125 * R.card) + 0.0025 * L.card) + out
        nl = (base + (0.0025 * L.card) * R.card) + out
        if hj <= nl:
            cands.append((hj, L.rels, OP_HASH, L, R))
        else:
            cands.append((nl, L.rels, OP_NESTLOOP, L, R))
    c, _, op, L, R = min(cands, key=lambda t: (t[0], t[1], t[2]))
    return Node(S, c, cS, op, L, R)


# ------------------------------------------------------------------ exact step on units

def unit_query(G: Graph, units: list[tuple[int, object]], cm: int, cache=None):
    """H3: the query over `units` (relation set, plan), labelled by lowest relation."""
    from paper_2202_13511_amd.workloads import Query
    order = sorted(range(len(units)), key=lambda i: lowest(units[i][0]))
    us = [units[i] for i in order]
    where = {}
    for i, (S, _) in enumerate(us):
        T = S
        while T:
            v = lowest(T)
            where[v] = i
            T &= T - 1
    cross = {}
    for (a, b), s in zip(G.edges, G.sel):
        if a in where and b in where and where[a] != where[b]:
            i, j = sorted((where[a], where[b]))
            cross[(i, j)] = cross.get((i, j), 1.0) * s
    keys = sorted(cross)
    edges = np.array(keys, dtype=np.uint32).reshape(-1, 2)
    sel = np.array([max(cross[e], DBL_MIN) for e in keys], dtype=np.float64)
    card = np.array([G.card_of(S) for S, _ in us], dtype=np.float64)
    bc = np.array([recost(G, p, cm, cache).cost for _, p in us], dtype=np.float64)
    return Query(len(us), edges, card, sel, "units", base_cost=bc), us


def exact_units(G: Graph, units, cm: int, cache=None):
    """Plan `units` with the oracle's MPDP; returns the expanded plan."""
    if len(units) == 1:
        return units[0][1]
    q, us = unit_query(G, units, cm, cache)
    memo = oracle.mpdp(q, cm)

    def build(S: int):
        if S & (S - 1) == 0:
            return us[lowest(S)][1]
        L = int(memo.left[S])
        return ("join", build(L), build(S & ~L))

    return build(memo.full)


def exact(q, cm: int):
    """Exact MPDP over the whole query (n <= 30), as a plan."""
    G = Graph(q)
    return exact_units(G, [(1 << v, ("leaf", v)) for v in range(q.n)], cm)


# ------------------------------------------------------------------ GOO

def goo(q, cm: int = COUT):
    """H4: greedy operator ordering over connected trees."""
    G = Graph(q)
    trees = {v: (1 << v, ("leaf", v)) for v in range(q.n)}  # keyed by lowest relation
    while len(trees) > 1:
        best = None
        keys = sorted(trees)
        for i in keys:
            Si = trees[i][0]
            nb = 0
            T = Si
            while T:
                nb |= G.adj[lowest(T)]
                T &= T - 1
            for j in keys:
                if j <= i or not (nb & trees[j][0]):
                    continue
                c = G.card_of(Si | trees[j][0])
                key = (c, i, j)
                if best is None or key < best:
                    best = key
        if best is None:
            raise ValueError("join graph is not connected")
        _, i, j = best
        Si, Pi = trees.pop(i)
        Sj, Pj = trees.pop(j)
        trees[min(i, j)] = (Si | Sj, ("join", Pi, Pj))
    return next(iter(trees.values()))[1]


# ------------------------------------------------------------------ IDP2

def idp2(q, k: int, cm: int = COUT, initial=None, trace=None):
    """Section 4.1: IDP2 with GOO's plan as the initial tree (H5).  With
    `trace` (a list), the relation set of every re-planned subtree is
    appended in the order IDP2 picks them."""
    G = Graph(q)
    cache = {}
    # tree over units: a unit is ("unit", relset, plan); a join ("join", A, B)
    def to_units(p):
        if p[0] == "leaf":
            return ("unit", 1 << p[1], p)
        return ("join", to_units(p[1]), to_units(p[2]))

    T = to_units(initial if initial is not None else goo(q, cm))

    def expand(t):
        if t[0] == "unit":
            return t[2]
        return ("join", expand(t[1]), expand(t[2]))

    while T[0] != "unit":
        # every subtree: (units, cost, lowest relation, path)
        best = None

        def visit(t, path):
            nonlocal best
            if t[0] == "unit":
                return [t], t[1]
            ua, Sa = visit(t[1], path + (1,))
            ub, Sb = visit(t[2], path + (2,))
            us = ua + ub
            if 2 <= len(us) <= k:
                c = recost(G, expand(t), cm, cache).cost
                key = (-c, lowest(Sa | Sb))
                if best is None or key < best[0]:
                    best = (key, path, us)
            return us, Sa | Sb

        visit(T, ())
        _, path, us = best
        plan = exact_units(G, [(u[1], u[2]) for u in us], cm, cache)
        S = 0
        for u in us:
            S |= u[1]
        if trace is not None:
            trace.append(S)
        new = ("unit", S, plan)

        def replace(t, p):
            if not p:
                return new
            if p[0] == 1:
                return ("join", replace(t[1], p[1:]), t[2])
            return ("join", t[1], replace(t[2], p[1:]))

        T = replace(T, path)
    return T[2]


# ------------------------------------------------------------------ UnionDP

def unit_edges(G: Graph, units: list):
    """Edges between units (sorted by lowest relation): sorted pairs (i, j),
    i < j, with the number of base edges and the product of their
    selectivities in edge-list order."""
    where = {}
    for i, (S, _) in enumerate(units):
        T = S
        while T:
            where[lowest(T)] = i
            T &= T - 1
    info = {}
    for (a, b), s in zip(G.edges, G.sel):
        if where[a] != where[b]:
            key = tuple(sorted((where[a], where[b])))
            cnt, prod = info.get(key, (0, 1.0))
            info[key] = (cnt + 1, prod * s)
    keys = sorted(info)
    return keys, [info[k_][0] for k_ in keys], [info[k_][1] for k_ in keys]


def partition(G: Graph, units: list, k: int) -> list[list]:
    """H6, the partition phase of Alg. 4 over `units` (sorted by lowest
    relation): groups of units, each connected and of at most k units; edges
    by (current size of both parts, weight, edge order), re-keyed as parts
    grow."""
    uedges, _, _ = unit_edges(G, units)
    parent = list(range(len(units)))
    size = [1] * len(units)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    def union(ri, rj):
        lo, hi = min(ri, rj), max(ri, rj)
        parent[hi] = lo
        size[lo] += size[hi]

    weight = [G.card_of(units[i][0] | units[j][0]) for i, j in uedges]
    heap = [(2, weight[e], e) for e in range(len(uedges))]
    heapq.heapify(heap)
    while heap:
        s, w, e = heapq.heappop(heap)
        i, j = uedges[e]
        ri, rj = find(i), find(j)
        if ri == rj:
            continue
        cur = size[ri] + size[rj]
        if cur > k:
            continue  # sizes only grow: this edge never joins two partitions again
        if cur != s:
            heapq.heappush(heap, (cur, w, e))  # re-keyed: the partitions have grown
            continue
        union(ri, rj)
    groups = {}
    for i in range(len(units)):
        groups.setdefault(find(i), []).append(units[i])
    return [groups[r] for r in sorted(groups)]


FEATURES = 32


def part_features(G: Graph, units: list, parts: list, pairs: list, cm: int, cache=None) -> np.ndarray:
    """L1: features of candidate unions of two parts (parts are lists of unit
    indices; pairs (a, b), a < b, index parts), float64, then rounded to
    float32 and to bfloat16 (bit patterns).  For parts A, B with weight
    w = card(A u B), each pair put as (smaller, larger):
      0,1  log10 card(A), card(B)                 / 8
      2    log10 w                                 / 8
      3    (log10 w - log10 card(A) - log10 card(B)) / 8
      4,5  log10(1 + summed plan cost of the units of A, of B) / 8
      6,7  log2 of the relations of A, B          / 4
      8,9  candidate unions of A, B               / 8
      10,11 units of A, B                         / 8
      12,13 share of A's (B's) candidates with a smaller weight than w
      14,15 log10 w - log10 of the smallest weight of a candidate of A (B), / 8
      16   log2 of the parts                       / 12
      17   share of all candidates with a smaller weight than w
      18   1
    the rest 0."""
    from oracle import mlp
    rels = []
    for p in parts:
        S = 0
        for u in p:
            S |= units[u][0]
        rels.append(S)
    card = [G.card_of(S) for S in rels]
    ucost = [recost(G, pl, cm, cache).cost for _, pl in units]
    cost = []
    for p in parts:
        c = 0.0
        for u in p:
            c = c + ucost[u]
        cost.append(c)
    w = [G.card_of(rels[a] | rels[b]) for a, b in pairs]
    inc = {}
    for e, (a, b) in enumerate(pairs):
        inc.setdefault(a, []).append(w[e])
        inc.setdefault(b, []).append(w[e])
    F = np.zeros((len(pairs), FEATURES), np.float64)
    for e, (a, b) in enumerate(pairs):
        lw = math.log10(w[e])
        la, lb = math.log10(card[a]), math.log10(card[b])
        pa, pb = math.log10(1.0 + cost[a]), math.log10(1.0 + cost[b])
        na, nb = math.log2(bin(rels[a]).count("1")), math.log2(bin(rels[b]).count("1"))
        da, db = len(inc[a]), len(inc[b])
        ua, ub = len(parts[a]), len(parts[b])
        ra = sum(1 for x in inc[a] if x < w[e]) / da
        rb = sum(1 for x in inc[b] if x < w[e]) / db
        ma = lw - math.log10(min(inc[a]))
        mb = lw - math.log10(min(inc[b]))
        g = sum(1 for x in w if x < w[e]) / len(w)
        F[e, 0], F[e, 1] = min(la, lb) / 8, max(la, lb) / 8
        F[e, 2] = lw / 8
        F[e, 3] = (lw - la - lb) / 8
        F[e, 4], F[e, 5] = min(pa, pb) / 8, max(pa, pb) / 8
        F[e, 6], F[e, 7] = min(na, nb) / 4, max(na, nb) / 4
        F[e, 8], F[e, 9] = min(da, db) / 8, max(da, db) / 8
        F[e, 10], F[e, 11] = min(ua, ub) / 8, max(ua, ub) / 8
        F[e, 12], F[e, 13] = min(ra, rb), max(ra, rb)
        F[e, 14], F[e, 15] = min(ma, mb) / 8, max(ma, mb) / 8
        F[e, 16] = math.log2(len(parts)) / 12
        F[e, 17] = g
        F[e, 18] = 1.0
    return mlp.bf16_bits(F)


ONE_PER_PASS = True


def learned_partition(G: Graph, units: list, k: int, cm: int, score, cache=None, examples=None, plan_sets=None,
                      one_per_pass=ONE_PER_PASS):
    """L2: the learned partition phase over `units` (sorted by lowest
    relation).  Parts start as single units.  Each pass scores every union
    of two adjacent parts with at most k units together (pairs of part
    indices ascending, parts numbered by their lowest unit), then joins the
    best-scored candidate (ties by pair order) if its score is positive
    (one_per_pass=False: every positive candidate, by decreasing score, whose
    parts no earlier join of the pass touched); passes repeat until none
    joins.  Returns the groups, or None when the first
    pass joins nothing (the caller then uses the paper's order, L4).  With
    `examples`, every pass appends (features, labels) (L3)."""
    where = {}
    for i, (S, _) in enumerate(units):
        T = S
        while T:
            where[lowest(T)] = i
            T &= T - 1
    uedges = sorted({tuple(sorted((where[a], where[b]))) for a, b in G.edges if where[a] != where[b]})
    parts = [[i] for i in range(len(units))]
    owner = list(range(len(units)))
    joined = False
    while True:
        pairs = sorted({tuple(sorted((owner[i], owner[j]))) for i, j in uedges
                        if owner[i] != owner[j] and len(parts[owner[i]]) + len(parts[owner[j]]) <= k})
        if not pairs:
            break
        X = part_features(G, units, parts, pairs, cm, cache)
        if examples is not None:
            rel = []
            for p in parts:
                S = 0
                for u in p:
                    S |= units[u][0]
                rel.append(S)
            examples.append((X, np.array([1.0 if (rel[a] | rel[b]) in plan_sets else 0.0 for a, b in pairs])))
        s = score(X)
        touched = set()
        did = False
        for e in sorted(range(len(pairs)), key=lambda e: (-s[e], e)):
            if not s[e] > 0:
                break
            a, b = pairs[e]
            if a in touched or b in touched:
                continue
            parts[a] = parts[a] + parts[b]
            parts[b] = []
            touched.add(a)
            touched.add(b)
            did = True
            if one_per_pass:
                break
        if not did:
            break
        joined = True
        parts = [sorted(p) for p in sorted((p for p in parts if p), key=min)]
        for pi, p in enumerate(parts):
            for u in p:
                owner[u] = pi
    if not joined:
        return None
    return [[units[u] for u in p] for p in parts]


def uniondp(q, k: int, cm: int = COUT, scorer=None, examples=None, plan_sets=None, teacher=False):
    """Section 4.2, Alg. 4 (H6).  With `scorer` (features -> one score per
    candidate union), the learned partition phase (L2), falling back to the
    paper's order for a round in which it joins nothing (L4).  teacher=True
    scores a candidate +1 if its union is one of `plan_sets` (the nodes of an
    optimal plan) and -1 otherwise.  With `examples`, the learned passes
    append (features, labels) (L3)."""
    G = Graph(q)
    cache = {}
    units = [(1 << v, ("leaf", v)) for v in range(q.n)]
    if teacher:
        last = []
        buf = examples if examples is not None else []

        def scorer(X, buf=buf):
            return buf[-1][1] * 2.0 - 1.0
        examples = buf
    while len(units) > k:
        units = sorted(units, key=lambda u: lowest(u[0]))
        groups = None
        if scorer is not None:
            groups = learned_partition(G, units, k, cm, scorer, cache, examples, plan_sets)
        if groups is None:
            groups = partition(G, units, k)
        nxt = []
        for members in groups:
            S = 0
            for m_ in members:
                S |= m_[0]
            nxt.append((S, exact_units(G, members, cm, cache)))
        units = nxt
    return exact_units(G, units, cm, cache)


def report(q, plan, cm: int):
    """(cost, flat plan) of a plan re-costed over the base relations (H2).
    Flat plan: nodes 0..n-1 are the relations, joins follow in post-order
    (left child first), the root is last; each node has left, right, rel
    (the relation, or the lowest relation below a join), nrels, op, cost and
    card."""
    G = Graph(q)
    root = recost(G, plan, cm, {})
    out = [dict(left=-1, right=-1, rel=v, nrels=1, op=OP_SCAN, cost=G.scan_cost(v, cm), card=G.card[v])
           for v in range(G.n)]

    def walk(nd: Node) -> int:
        if nd.left is None:
            return lowest(nd.rels)
        li = walk(nd.left)
        ri = walk(nd.right)
        out.append(dict(left=li, right=ri, rel=lowest(nd.rels), nrels=bin(nd.rels).count("1"), op=nd.op,
                        cost=nd.cost, card=nd.card))
        return len(out) - 1

    walk(root)
    return root.cost, out
