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
"""
from __future__ import annotations

import heapq
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

def idp2(q, k: int, cm: int = COUT, initial=None):
    """Section 4.1: IDP2 with GOO's plan as the initial tree (H5)."""
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

def partition(G: Graph, units: list, k: int) -> list[list]:
    """H6, the partition phase of Alg. 4 over `units` (sorted by lowest
    relation): groups of units, each connected and of at most k units."""
    where = {}
    for i, (S, _) in enumerate(units):
        T = S
        while T:
            where[lowest(T)] = i
            T &= T - 1
    uedges = sorted({tuple(sorted((where[a], where[b]))) for a, b in G.edges if where[a] != where[b]})
    weight = [G.card_of(units[i][0] | units[j][0]) for i, j in uedges]
    parent = list(range(len(units)))
    size = [1] * len(units)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

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
        lo, hi = min(ri, rj), max(ri, rj)
        parent[hi] = lo
        size[lo] += size[hi]
    groups = {}
    for i in range(len(units)):
        groups.setdefault(find(i), []).append(units[i])
    return [groups[r] for r in sorted(groups)]


def uniondp(q, k: int, cm: int = COUT):
    """Section 4.2, Alg. 4 (H6)."""
    G = Graph(q)
    cache = {}
    units = [(1 << v, ("leaf", v)) for v in range(q.n)]
    while len(units) > k:
        units = sorted(units, key=lambda u: lowest(u[0]))
        nxt = []
        for members in partition(G, units, k):
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
