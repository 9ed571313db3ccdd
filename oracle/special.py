"""Textbook special cases of the join-order DP (test oracle).

TEST INFRASTRUCTURE ONLY.

chain_interval_dp  On a chain 0-1-...-(n-1) the connected sets are the
                   intervals [i..j] and the csg-cmp pairs of [i..j] are the
                   splits [i..m] | [m+1..j]; the optimum is the O(n^3)
                   interval DP (matrix-chain style).
star_sorted_plan   On a star under C_out every plan joins one leaf at a time
                   onto the hub side, so the cost is the sum of the prefix
                   cardinalities; by an exchange argument the optimum adds the
                   leaves in ascending order of card[l] * sel(hub, l).

Both use the written definitions of card(S), C_out, the PG-like model and
the plan key stated in the header of mpdp_oracle.c.
"""
from __future__ import annotations

COST_COUT = 0
COST_PGLIKE = 1
OP_SCAN, OP_HASH, OP_NESTLOOP, OP_JOIN = 0, 1, 2, 3


def _interval_card(card, sel_next, i, j):
    """card(S) for S = {i..j} on a chain: v ascending, each v after the first
    multiplies its own card and then sel(v-1, v)."""
    c = 1.0
    for v in range(i, j + 1):
        c = c * card[v]
        if v > i:
            c = c * sel_next[v - 1]
    return 1.0 if c < 1.0 else c


def chain_interval_dp(q, cost_model=COST_COUT):
    """Return {interval bitmap: (cost, card, left bitmap, op)} for a chain
    whose edges are (i, i+1)."""
    n = q.n
    edges = q.edges.tolist()
    sel_next = [0.0] * max(n - 1, 0)
    for (u, v), s in zip(edges, q.sel.tolist()):
        a, b = min(u, v), max(u, v)
        if b != a + 1:
            raise ValueError("not a chain labelled 0..n-1")
        sel_next[a] = float(s)
    card = [float(c) for c in q.card.tolist()]

    def bm(i, j):
        return ((1 << (j + 1)) - 1) & ~((1 << i) - 1)

    best = {}
    for v in range(n):
        best[bm(v, v)] = (0.01 * card[v] if cost_model == COST_PGLIKE else 0.0, card[v], 0, OP_SCAN)
    for length in range(2, n + 1):
        for i in range(0, n - length + 1):
            j = i + length - 1
            cS = _interval_card(card, sel_next, i, j)
            cand = []
            for m in range(i, j):
                A, B = bm(i, m), bm(m + 1, j)
                for L, R in ((A, B), (B, A)):
                    cL, kL = best[L][0], best[L][1]
                    cR, kR = best[R][0], best[R][1]
                    if cost_model == COST_COUT:
                        cand.append(((cL + cR) + cS, L, OP_JOIN))
                    else:
                        hj = (((cL + cR) + 0.0125 * kR) + 0.0025 * kL) + 0.01 * cS
                        nl = ((cL + cR) + (0.0025 * kL) * kR) + 0.01 * cS
                        cand.append((hj, L, OP_HASH) if hj <= nl else (nl, L, OP_NESTLOOP))
            c, L, op = min(cand)
            best[bm(i, j)] = (c, cS, L, op)
    return best


def star_sorted_plan(q):
    """Leaf order and C_out cost of the ascending card*sel plan on a star
    with hub 0.  Returns (order, cost, any_prefix_clamped)."""
    n = q.n
    card = [float(c) for c in q.card.tolist()]
    sel = {}
    for (u, v), s in zip(q.edges.tolist(), q.sel.tolist()):
        if min(u, v) != 0:
            raise ValueError("not a star with hub 0")
        sel[max(u, v)] = float(s)
    order = sorted(range(1, n), key=lambda l: (card[l] * sel[l], l))

    def card_of(S):
        c = 1.0
        for v in range(n):
            if S >> v & 1:
                c = c * card[v]
                if v > 0 and (S & 1):
                    c = c * sel[v]
        return (1.0 if c < 1.0 else c), c < 1.0

    cost = 0.0
    S = 1
    clamped = False
    for leaf in order:
        S |= 1 << leaf
        cS, cl = card_of(S)
        clamped = clamped or cl
        cost = (cost + 0.0) + cS
    return order, cost, clamped
