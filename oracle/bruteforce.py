"""Brute force over every cross-product-free bushy join tree (test oracle).

TEST INFRASTRUCTURE ONLY.  This is the plain definition of the optimum the
paper's DP algorithms reach (Section 2.1 objective, theorems of Section 3):
the minimum cost over all join trees whose every inner node joins a
csg-cmp pair (the four conditions of Section 2.1).  Every tree is built
explicitly; nothing is pruned, so the cost lists grow as the number of trees
(n! * Catalan(n-1) ordered trees for an n-clique).

It is written independently of mpdp_oracle.c (pure Python floats, which are
IEEE doubles rounded to nearest) and uses the same written definitions of
card(S), C_out and the PG-like model (see the header of mpdp_oracle.c).
"""
from __future__ import annotations

COST_COUT = 0
COST_PGLIKE = 1


def _graph(q):
    n = q.n
    adj = [0] * n
    sel = {}
    for (u, v), s in zip(q.edges.tolist(), q.sel.tolist()):
        adj[u] |= 1 << v
        adj[v] |= 1 << u
        sel[(min(u, v), max(u, v))] = float(s)
    return n, adj, sel, [float(c) for c in q.card.tolist()]


def bruteforce(q, cost_model=COST_COUT):
    """Return (minimum cost, number of trees enumerated, {set: min cost})."""
    n, adj, sel, card = _graph(q)
    if n > 7 or (cost_model == COST_PGLIKE and n > 6):
        raise ValueError("brute force is limited to n <= 7 (n <= 6 for PG-like)")

    def members(S):
        return [v for v in range(n) if S >> v & 1]

    def card_of(S):
        c = 1.0
        for v in members(S):
            c = c * card[v]
            for u in members(S):
                if u < v and (adj[v] >> u & 1):
                    c = c * sel[(u, v)]
        return 1.0 if c < 1.0 else c

    def connected(S):
        if S == 0:
            return False
        seen = S & -S
        while True:
            grown = seen
            for v in members(seen):
                grown |= adj[v] & S
            if grown == seen:
                return seen == S
            seen = grown

    def adjacent(A, B):
        return any(adj[v] & B for v in members(A))

    lists = {}

    def trees(S):
        if S in lists:
            return lists[S]
        if S & (S - 1) == 0:
            v = S.bit_length() - 1
            out = [0.01 * card[v] if cost_model == COST_PGLIKE else 0.0]
        else:
            cS = card_of(S)
            out = []
            L = (S - 1) & S
            while L:
                R = S & ~L
                if connected(L) and connected(R) and adjacent(L, R):
                    kL, kR = card_of(L), card_of(R)
                    for a in trees(L):
                        for b in trees(R):
                            if cost_model == COST_COUT:
                                out.append((a + b) + cS)
                            else:
                                out.append((((a + b) + 0.0125 * kR) + 0.0025 * kL) + 0.01 * cS)
                                out.append(((a + b) + (0.0025 * kL) * kR) + 0.01 * cS)
                L = (L - 1) & S
        lists[S] = out
        return out

    full = (1 << n) - 1
    allc = trees(full)
    return min(allc), len(allc), {S: min(v) for S, v in lists.items() if v}
