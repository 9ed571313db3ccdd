"""Pins of the large-query heuristics oracle (oracle/heuristics.py, Section 4).

  * with k >= n, IDP2 and UnionDP hand the whole query to the exact step, so
    both must reach the exact DP's optimum bit for bit; the re-costing of the
    exact plan must reproduce the DP's root cost bit for bit;
  * IDP2 only ever replaces a subtree by the optimal plan of the same units,
    so it can never end above its GOO start;
  * every heuristic returns a plan whose joins split a connected set into two
    disjoint, connected, adjacent parts and whose leaves are the relations;
  * GOO and the UnionDP partition phase on examples worked by hand;
  * the unit query of single relations is the query itself.
"""
import numpy as np
import pytest

import oracle
from oracle import heuristics as H
from paper_2202_13511_amd import workloads as W

CMS = [oracle.COST_COUT, oracle.COST_PGLIKE]


def small_queries():
    return [W.snowflake(14, 3), W.cycle_chords(2, n=12, chords=3), W.random_connected(11, 5, 0.25),
            W.star(10, 1), W.chain(12, 2)]


def leaves(plan):
    if plan[0] == "leaf":
        return [plan[1]]
    return leaves(plan[1]) + leaves(plan[2])


def check_plan(q, plan):
    G = H.Graph(q)
    assert sorted(leaves(plan)) == list(range(q.n))

    def rels(p):
        if p[0] == "leaf":
            return 1 << p[1]
        a, b = rels(p[1]), rels(p[2])
        assert a & b == 0
        for X in (a, b):  # each side induces a connected subgraph
            seen, fr = X & -X, X & -X
            while fr:
                nb = 0
                T = fr
                while T:
                    nb |= G.adj[H.lowest(T)]
                    T &= T - 1
                fr = nb & X & ~seen
                seen |= fr
            assert seen == X
        T, nb = a, 0
        while T:
            nb |= G.adj[H.lowest(T)]
            T &= T - 1
        assert nb & b, "the two sides are not adjacent"
        return a | b

    assert rels(plan) == (1 << q.n) - 1


@pytest.mark.parametrize("cm", CMS)
def test_whole_query_reaches_exact_optimum(cm):
    for q in small_queries():
        ex = oracle.mpdp(q, cm).root_cost
        c, nodes = H.report(q, H.exact(q, cm), cm)
        assert np.float64(c).view(np.uint64) == np.float64(ex).view(np.uint64), q.name
        assert len(nodes) == 2 * q.n - 1
        for f in (H.uniondp, H.idp2):
            c2, _ = H.report(q, f(q, q.n, cm), cm)
            assert np.float64(c2).view(np.uint64) == np.float64(ex).view(np.uint64), (q.name, f.__name__)


@pytest.mark.parametrize("cm", CMS)
def test_heuristics_valid_and_idp2_improves_goo(cm):
    qs = small_queries() + [W.large_snowflake(60, 3), W.large_snowflake(90, 4)]
    for q in qs:
        g = H.goo(q, cm)
        check_plan(q, g)
        cg, _ = H.report(q, g, cm)
        for k in (3, 5, 8):
            p = H.idp2(q, k, cm)
            check_plan(q, p)
            ci, _ = H.report(q, p, cm)
            assert ci <= cg * (1 + 1e-12), (q.name, k)
            u = H.uniondp(q, k, cm)
            check_plan(q, u)
        if q.n <= 14:
            ex = oracle.mpdp(q, cm).root_cost
            for k in (3, 5, 8):
                ci, _ = H.report(q, H.idp2(q, k, cm), cm)
                cu, _ = H.report(q, H.uniondp(q, k, cm), cm)
                assert ci >= ex * (1 - 1e-12) and cu >= ex * (1 - 1e-12)


def test_goo_by_hand():
    """Chain 0-1-2-3, cards (10, 1000, 100, 10000), sels 0.001, 0.01, 1e-4.
    Two-relation joins: {0,1} = 10, {1,2} = 1000, {2,3} = 100: GOO joins
    {0,1}; then {0,1,2} = 10 beats {2,3} = 100; then the last join.  C_out
    = 10 + 10 + 10 = 30."""
    q = W.Query(4, np.array([[0, 1], [1, 2], [2, 3]], np.uint32), np.array([10.0, 1000.0, 100.0, 10000.0]),
                np.array([0.001, 0.01, 1e-4]))
    p = H.goo(q)
    assert p == ("join", ("join", ("join", ("leaf", 0), ("leaf", 1)), ("leaf", 2)), ("leaf", 3))
    c, _ = H.report(q, p, oracle.COST_COUT)
    assert abs(c - 30.0) < 1e-9


def test_uniondp_partition_by_hand():
    """Chain 0-..-5, all cards 10, sels (0.05, 0.01, 0.07, 0.02, 0.03):
    weights 5, 1, 7, 2, 3.  With k = 2 the edges go by (size, weight):
    (1,2) w=1 joins; (3,4) w=2 joins; (4,5), (0,1), (2,3) would exceed 2."""
    q = W.Query(6, np.array([[i, i + 1] for i in range(5)], np.uint32), np.full(6, 10.0),
                np.array([0.05, 0.01, 0.07, 0.02, 0.03]))
    G = H.Graph(q)
    units = [(1 << v, ("leaf", v)) for v in range(6)]
    groups = H.partition(G, units, 2)
    sets = [sum(u[0] for u in g) for g in groups]
    assert sets == [0b000001, 0b000110, 0b011000, 0b100000]
    # k = 3: (1,2) w=1; (3,4) w=2; then (4,5): 2 + 1 = 3 joins; (0,1): 1 + 2 = 3 joins
    groups = H.partition(G, units, 3)
    assert [sum(u[0] for u in g) for g in groups] == [0b000111, 0b111000]


@pytest.mark.parametrize("k", [4, 7, 12])
def test_partition_invariants(k):
    q = W.large_snowflake(120, 7)
    G = H.Graph(q)
    units = [(1 << v, ("leaf", v)) for v in range(q.n)]
    groups = H.partition(G, units, k)
    cover = 0
    for g in groups:
        S = sum(u[0] for u in g)
        assert cover & S == 0
        cover |= S
        assert 1 <= len(g) <= k
        # connected
        seen, fr = S & -S, S & -S
        while fr:
            nb = 0
            T = fr
            while T:
                nb |= G.adj[H.lowest(T)]
                T &= T - 1
            fr = nb & S & ~seen
            seen |= fr
        assert seen == S
    assert cover == (1 << q.n) - 1
    assert max(len(g) for g in groups) >= 2


def test_unit_query_of_single_relations_is_the_query():
    q = W.cycle_chords(4, n=10, chords=3)
    G = H.Graph(q)
    uq, _ = H.unit_query(G, [(1 << v, ("leaf", v)) for v in range(q.n)], oracle.COST_PGLIKE)
    order = np.lexsort((q.edges[:, 1], q.edges[:, 0]))
    assert np.array_equal(uq.edges, q.edges[order])
    assert np.array_equal(uq.sel.view(np.uint64), q.sel[order].view(np.uint64))
    assert np.array_equal(uq.card.view(np.uint64), q.card.view(np.uint64))
    assert np.array_equal(uq.base_cost, 0.01 * q.card)


def _leaf(v):
    return ("leaf", v)


def _join(a, b):
    return ("join", a, b)


IDP2_CHAIN = dict(edges=[[0, 1], [1, 2], [2, 3], [3, 4]], card=[4.0, 4.0, 4.0, 64.0, 64.0],
                  sel=[0.5, 0.5, 0.25, 0.5])


def idp2_chain():
    return W.Query(5, np.array(IDP2_CHAIN["edges"], np.uint32), np.array(IDP2_CHAIN["card"]),
                   np.array(IDP2_CHAIN["sel"]))


def test_idp2_replans_the_costliest_subtree_by_hand():
    """Section 4.1: IDP2 re-plans the subtree T' with 1 < |T'| <= k units of
    maximal cost C(T').  Chain 0-1-2-3-4, cards (4, 4, 4, 64, 64), sels
    (0.5, 0.5, 0.25, 0.5), C_out, k = 3, all values exact in binary:
      card{0,1} = card{1,2} = 8, card{0,1,2} = 16, card{3,4} = 2048,
      card{0,1,2,3} = 256, card of all = 8192.
    From the tree ((0 1) 2) (3 4): the 2..3-unit subtrees cost (0 1) = 8,
    ((0 1) 2) = 8 + 16 = 24, (3 4) = 2048.  The costliest is (3 4), which is
    neither the first one met nor the cheapest.  Then ((0 1) 2) = 24 beats
    (0 1) = 8; its exact plan ties 24 = 24 between (0 1) 2 and 0 (1 2), and
    the smaller left set {0} wins: 0 (1 2).  Last the two units.  Result
    (0 (1 2)) (3 4), cost 24 + 2048 + 8192 = 10264.
    From GOO's tree (GOO: {0,1} = 8 ties {1,2} = 8 and the smaller lowest
    relations win; then {0,1,2} = 16, {0,1,2,3} = 256, then 4): the
    candidates are (0 1) = 8 and ((0 1) 2) = 24, so {0,1,2} is re-planned to
    0 (1 2); then the root (3 units, 24 + 256 + 8192 = 8472) beats
    (U 3) = 280; its exact plan over U = {0,1,2}, 3, 4 compares
    U (3 4) = 24 + 2048 + 8192 = 10264 with (U 3) 4 = 24 + 256 + 8192 = 8472.
    Picking the cheapest or the first subtree re-plans {0,1} first and keeps
    (0 1) 2 instead."""
    q = idp2_chain()
    initial = _join(_join(_join(_leaf(0), _leaf(1)), _leaf(2)), _join(_leaf(3), _leaf(4)))
    trace = []
    p = H.idp2(q, 3, oracle.COST_COUT, initial=initial, trace=trace)
    assert trace == [0b11000, 0b00111, 0b11111]
    assert p == _join(_join(_leaf(0), _join(_leaf(1), _leaf(2))), _join(_leaf(3), _leaf(4)))
    c, _ = H.report(q, p, oracle.COST_COUT)
    assert c == 10264.0

    assert H.goo(q) == _join(_join(_join(_join(_leaf(0), _leaf(1)), _leaf(2)), _leaf(3)), _leaf(4))
    trace = []
    p = H.idp2(q, 3, oracle.COST_COUT, trace=trace)
    assert trace == [0b00111, 0b11111]
    assert p == _join(_join(_join(_leaf(0), _join(_leaf(1), _leaf(2))), _leaf(3)), _leaf(4))
    c, _ = H.report(q, p, oracle.COST_COUT)
    assert c == 8472.0


UNION_LADDER = dict(edges=[[0, 1], [1, 2], [2, 3], [0, 3], [3, 4], [4, 5]], card=[8.0] * 6,
                    sel=[0.125, 0.5, 0.125, 0.25, 0.1875, 0.125])


def union_ladder():
    return W.Query(6, np.array(UNION_LADDER["edges"], np.uint32), np.array(UNION_LADDER["card"]),
                   np.array(UNION_LADDER["sel"]))


def test_uniondp_composite_edge_multiplies_its_selectivities_by_hand():
    """Alg. 4 (composite nodes) with H3: two units joined by several base
    edges get one edge whose selectivity is the product of theirs.
    Relations 0..5, all cards 8, edges (0,1) 0.125, (1,2) 0.5, (2,3) 0.125,
    (0,3) 0.25, (3,4) 0.1875, (4,5) 0.125; C_out, k = 3.
    Partition: the weights of (0,1), (2,3), (4,5) are 8*8*0.125 = 8, the
    others 32, 16, 12; the three pairs join first and every other union
    would hold 4 > 3 units.  Units U0 = {0,1}, U1 = {2,3}, U2 = {4,5}, cards
    8, base costs 8.  The unit query's edges: U0-U1 through (1,2) and (0,3),
    selectivity 0.5 * 0.25 = 0.125; U1-U2 through (3,4), 0.1875.
    Exact step: (U0 U1) U2 pays card(U0 u U1) = 8*8*0.125 = 8, U0 (U1 U2)
    pays 8*8*0.1875 = 12: the first wins.  With only the first selectivity
    (0.5 -> 32), only the second (0.25 -> 16), their sum or their minimum,
    the other plan would win.  Re-costed over the base relations:
    card{0,1,2,3} = 8, card of all = 12, cost 8 + 8 + 8 + 8 + 12 = 44."""
    q = union_ladder()
    G = H.Graph(q)
    units = [(1 << v, _leaf(v)) for v in range(6)]
    groups = H.partition(G, units, 3)
    assert [sum(u[0] for u in g) for g in groups] == [0b000011, 0b001100, 0b110000]
    uq, _ = H.unit_query(G, [(0b000011, _join(_leaf(0), _leaf(1))), (0b001100, _join(_leaf(2), _leaf(3))),
                             (0b110000, _join(_leaf(4), _leaf(5)))], oracle.COST_COUT)
    assert uq.edges.tolist() == [[0, 1], [1, 2]]
    assert uq.sel.tolist() == [0.125, 0.1875]
    assert uq.card.tolist() == [8.0, 8.0, 8.0] and uq.base_cost.tolist() == [8.0, 8.0, 8.0]
    p = H.uniondp(q, 3, oracle.COST_COUT)
    assert p == _join(_join(_join(_leaf(0), _leaf(1)), _join(_leaf(2), _leaf(3))), _join(_leaf(4), _leaf(5)))
    c, _ = H.report(q, p, oracle.COST_COUT)
    assert c == 44.0
