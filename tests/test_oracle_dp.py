"""DP pins of the CPU oracle: brute force, algorithm agreement, special cases.

  * brute force over every bushy tree (n <= 7) reaches the DP's root cost
    bit for bit, and every connected set's minimum;
  * DPSUB (Alg. 1), MPDP (Alg. 2/3) and the level-bucketed DPccp produce the
    same memo bit for bit;
  * the chain interval DP and the sorted star order (textbook special cases);
  * card(S) against its exact rational value; a two-relation example worked
    by hand from the written cost definitions.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.bruteforce import bruteforce
from oracle.special import chain_interval_dp, star_sorted_plan
from paper_2202_13511_amd import workloads as W

CMS = [oracle.COST_COUT, oracle.COST_PGLIKE]


def same_memo(a, b):
    ma, mb = a.has_plan(), b.has_plan()
    assert np.array_equal(ma, mb)
    assert np.array_equal(a.cost[ma].view(np.uint64), b.cost[mb].view(np.uint64))
    assert np.array_equal(a.card[ma].view(np.uint64), b.card[mb].view(np.uint64))
    assert np.array_equal(a.left[ma], b.left[mb])
    assert np.array_equal(a.op[ma], b.op[mb])


def small_graphs():
    out = []
    for s in range(3):
        out += [W.random_connected(9, s, 0.2), W.random_connected(10, 10 + s, 0.45),
                W.random_tree(11, s), W.cycle(8, s), W.clique(7, s), W.chain(9, s),
                W.star(10, s), W.snowflake(12, s), W.cycle_chords(s, n=11, chords=3)]
    out.append(W.all_equal_clique(7))
    return out


@pytest.mark.parametrize("cm", CMS)
def test_dp_algorithms_agree(cm):
    for q in small_graphs():
        d = oracle.dpsub(q, cm)
        same_memo(d, oracle.mpdp(q, cm))
        same_memo(d, oracle.mpdp(q, cm, force_general=True))
        same_memo(d, oracle.dpccp(q, cm))
        assert d.ccp_ordered == 2 * oracle.count_ccp(q)


@pytest.mark.parametrize("cm", CMS)
def test_threaded_levels_agree(cm):
    """The level loop split over threads (sets of one size depend only on
    smaller sets, Section 5) gives the same memo and counters as one thread,
    also where the split puts every set of a level in its own part (n < 10)."""
    qs = small_graphs()[:9] + [W.star(6, 0), W.cycle_chords(1, n=14, chords=5), W.clique(12, 2)]
    for q in qs:
        a = oracle.mpdp(q, cm)
        for t in (2, 5):
            b = oracle.mpdp(q, cm, threads=t)
            same_memo(a, b)
            assert (a.evaluated, a.ccp_ordered, a.connected_sets) == \
                (b.evaluated, b.ccp_ordered, b.connected_sets), q.name


@pytest.mark.parametrize("cm", CMS)
def test_bruteforce_matches_dp(cm):
    nmax = 7 if cm == oracle.COST_COUT else 6
    qs = [W.random_connected(nmax, s, 0.3) for s in range(4)] + \
         [W.clique(nmax, 1), W.star(nmax, 2), W.cycle(nmax, 3), W.chain(nmax, 4),
          W.all_equal_clique(nmax)]
    for q in qs:
        best, ntrees, per_set = bruteforce(q, cm)
        m = oracle.mpdp(q, cm)
        assert np.float64(best).view(np.uint64) == np.float64(m.root_cost).view(np.uint64), q.name
        for S, c in per_set.items():
            assert np.float64(c).view(np.uint64) == m.cost[S].view(np.uint64), (q.name, S)


def test_bruteforce_tree_count_clique():
    """An n-clique has n! * Catalan(n-1) ordered bushy trees."""
    for n in range(2, 8):
        _, ntrees, _ = bruteforce(W.clique(n, 0))
        assert ntrees == math.factorial(n) * math.comb(2 * (n - 1), n - 1) // n


def recost(q, plan, cm):
    """Re-cost a plan bottom-up from its own nodes."""
    card = {}
    cost = {}
    for i, nd in enumerate(plan):
        if nd["left"] < 0:
            v = nd["relset"].bit_length() - 1
            cost[i] = 0.01 * float(q.card[v]) if cm == oracle.COST_PGLIKE else 0.0
            card[i] = float(q.card[v])
        else:
            a, b = nd["left"], nd["right"]
            cS = oracle.card(q, nd["relset"])
            card[i] = cS
            if cm == oracle.COST_COUT:
                cost[i] = (cost[a] + cost[b]) + cS
            elif nd["op"] == oracle.OP_HASH:
                cost[i] = (((cost[a] + cost[b]) + 0.0125 * card[b]) + 0.0025 * card[a]) + 0.01 * cS
            else:
                cost[i] = ((cost[a] + cost[b]) + (0.0025 * card[a]) * card[b]) + 0.01 * cS
    return cost[len(plan) - 1]


@pytest.mark.parametrize("cm", CMS)
def test_plan_invariants(cm):
    for q in small_graphs():
        m = oracle.mpdp(q, cm)
        plan = oracle.plan_from_memo(m)
        assert len(plan) == 2 * q.n - 1
        assert plan[-1]["relset"] == (1 << q.n) - 1
        for nd in plan[q.n:]:
            L, R = plan[nd["left"]]["relset"], plan[nd["right"]]["relset"]
            assert L & R == 0 and L | R == nd["relset"]
            assert oracle.grow(q, L & -L, L) == L and oracle.grow(q, R & -R, R) == R
            assert oracle.grow(q, L, L | R) == L | R  # L adjacent to R
        assert recost(q, plan, cm) == m.root_cost


@pytest.mark.parametrize("cm", CMS)
def test_chain_interval_dp(cm):
    for n, seed in [(5, 0), (12, 1), (20, 2), (24, 3)]:
        q = W.chain(n, seed)
        m = oracle.mpdp(q, cm)
        ref = chain_interval_dp(q, cm)
        for S, (c, k, L, op) in ref.items():
            if S & (S - 1) == 0:
                continue
            assert m.cost[S] == c and m.card[S] == k and m.left[S] == L and m.op[S] == op, (n, S)


def test_star_sorted_order():
    """Under C_out the ascending card*sel order is optimal on a star."""
    for seed in range(8):
        q = W.star(14, seed)
        m = oracle.mpdp(q)
        order, cost, clamped = star_sorted_plan(q)
        assert m.root_cost <= cost
        assert (cost - m.root_cost) <= 1e-12 * cost
        if not clamped:
            # walk the DP plan: the leaf joined last sits at the top
            S, seq = (1 << q.n) - 1, []
            while S != 1:
                L = int(m.left[S])
                leaf = L if L & (L - 1) == 0 else S & ~L
                seq.append(leaf.bit_length() - 1)
                S &= ~leaf
            assert seq[::-1] == order


def test_card_matches_exact_product():
    """card(S) is the product of the cards of S and the selectivities of the
    edges inside S (clamped below at 1); the rounded value is within one
    rounding per multiplication of the exact rational product."""
    rng = np.random.Generator(np.random.PCG64(7))
    for q in [W.clique(10, 1), W.snowflake(16, 2), W.cycle_chords(3, n=14, chords=5)]:
        adj = q.adjacency()
        sel = {(min(u, v), max(u, v)): float(s) for (u, v), s in zip(q.edges.tolist(), q.sel.tolist())}
        for S in rng.integers(1, 1 << q.n, size=300).tolist():
            exact = Fraction(1)
            mults = 0
            for v in range(q.n):
                if S >> v & 1:
                    exact *= Fraction(float(q.card[v]))
                    mults += 1
                    for u in range(v):
                        if S >> u & 1 and adj[v] >> u & 1:
                            exact *= Fraction(sel[(u, v)])
                            mults += 1
            want = max(exact, Fraction(1))
            got = Fraction(oracle.card(q, S))
            if exact < 1:
                assert got == 1
            else:
                assert abs(got - want) <= want * Fraction(mults, 2 ** 52)


def test_two_relations_by_hand():
    """card = (100, 1000), sel = 0.001: card(S) = 100.
    C_out: 0 + 0 + 100 = 100.
    PG-like: base costs 1 and 10; HJ with {1} outer and {0} inner:
    11 + 0.0125*100 + 0.0025*1000 + 0.01*100 = 15.75, the cheapest of the four
    candidates (HJ other way 24.75, NL both ways 262)."""
    q = W.Query(2, np.array([[0, 1]], np.uint32), np.array([100.0, 1000.0]), np.array([0.001]))
    m = oracle.mpdp(q, oracle.COST_COUT)
    assert m.cost[3] == 100.0 and m.card[3] == 100.0 and m.left[3] == 1  # tie: lowest left
    m = oracle.mpdp(q, oracle.COST_PGLIKE)
    assert abs(m.cost[3] - 15.75) < 1e-12 and m.left[3] == 2 and m.op[3] == oracle.OP_HASH


def test_tie_storm_is_deterministic():
    q = W.all_equal_clique(8)
    a = oracle.mpdp(q)
    b = oracle.dpsub(q)
    same_memo(a, b)
    # with all statistics equal every split of S ties on cost; the smallest
    # left bitmap among the cheapest splits must be chosen
    assert int(a.left[(1 << 8) - 1]) & 1 == 1


@pytest.mark.parametrize("cm", CMS)
def test_induced_subquery_equals_memo_entry(cm):
    """The full-size cyclic checks solve a set S on its own induced sub-query
    (relations relabelled in increasing order).  That must reproduce the
    whole query's memo entry of S bit for bit, left set and operator included."""
    rng = np.random.Generator(np.random.PCG64(5))
    for q in [W.cycle_chords(3, n=14, chords=6), W.random_connected(13, 4, 0.3), W.snowflake(15, 1)]:
        m = oracle.mpdp(q, cm)
        mask = m.has_plan()
        conn = np.nonzero(mask)[0]
        conn = conn[conn & (conn - 1) != 0]
        for S in rng.choice(conn, size=40, replace=False).tolist():
            sub, rel = oracle.induced(q, S)
            ms = oracle.mpdp(sub, cm)
            assert ms.cost[ms.full] == m.cost[S] and ms.card[ms.full] == m.card[S]
            assert oracle.expand(rel, int(ms.left[ms.full])) == m.left[S]
            assert ms.op[ms.full] == m.op[S]


@pytest.mark.parametrize("cm", CMS)
def test_recost_plan_helper(cm):
    for q in small_graphs()[:9]:
        m = oracle.mpdp(q, cm)
        plan = oracle.plan_from_memo(m)
        assert oracle.recost_plan(q, plan, cm) == m.root_cost
        # a join node whose children do not cover it is rejected
        bad = [dict(nd) for nd in plan]
        bad[-1]["right"] = bad[-1]["left"]
        with pytest.raises(ValueError):
            oracle.recost_plan(q, bad, cm)
