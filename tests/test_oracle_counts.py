"""Counting pins of the CPU oracle: closed forms and the paper's printed ratios.

The oracle's counters are checked against mathematics that does not depend on
the oracle: closed-form numbers of csg-cmp pairs and connected sets for
chains, stars, cycles and cliques, and the evaluation ratios printed in the
paper (Section 2.3 / Figure 4 and Section 7.2.1).
"""
import json
import math
import os

import pytest

import oracle
from paper_2202_13511_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def ccp_closed_form(kind, n):
    """Unordered csg-cmp pair counts."""
    return {
        "chain": (n ** 3 - n) // 6,
        "star": (n - 1) * 2 ** (n - 2),
        "cycle": (n ** 3 - 2 * n ** 2 + n) // 2,
        "clique": (3 ** n - 2 ** (n + 1) + 1) // 2,
    }[kind]


def connected_closed_form(kind, n):
    """Connected subsets including singletons."""
    return {
        "chain": n * (n + 1) // 2,
        "star": 2 ** (n - 1) + n - 1,
        "cycle": n * (n - 1) + 1,
        "clique": 2 ** n - 1,
    }[kind]


GEN = {"chain": W.chain, "star": W.star, "cycle": W.cycle, "clique": W.clique}


@pytest.mark.parametrize("kind", ["chain", "star", "cycle", "clique"])
def test_closed_form_counts(kind):
    for n in range(3, 12):
        q = GEN[kind](n, 0)
        want = ccp_closed_form(kind, n)
        assert oracle.count_ccp(q) == want, (kind, n)
        d = oracle.dpsub(q)
        m = oracle.mpdp(q)
        assert d.ccp_ordered == 2 * want
        assert m.ccp_ordered == 2 * want
        assert d.connected_sets + n == connected_closed_form(kind, n)
        assert m.connected_sets + n == connected_closed_form(kind, n)


def test_closed_form_counts_larger():
    assert oracle.count_ccp(W.star(20, 0)) == ccp_closed_form("star", 20)
    assert oracle.count_ccp(W.chain(30, 0)) == ccp_closed_form("chain", 30)
    assert oracle.count_ccp(W.cycle(30, 0)) == ccp_closed_form("cycle", 30)
    assert oracle.count_ccp(W.clique(14, 0)) == ccp_closed_form("clique", 14)


def test_tree_pairs_per_set():
    """Section 3.1: a connected S of size i in a tree has exactly i-1 pairs, so
    the unordered pair count is the sum of (|S|-1) over connected sets."""
    for seed in range(6):
        q = W.random_tree(11, seed)
        m = oracle.mpdp(q)
        mask = m.has_plan()
        total = sum(bin(S).count("1") - 1 for S in range(1, 1 << q.n) if mask[S])
        assert oracle.count_ccp(q) == total
        assert m.ccp_ordered == 2 * total


def test_star_dpsub_gap_printed_ratio():
    """Figure 4 / Section 7.2.1: DPSUB's EvaluatedCounter is about 2805 times
    the CCP-Counter for a 25-relation star.  Alg. 1 evaluates every subset of
    every connected S, i.e. 2 * (3^(n-1) - 1) over the sets with |S| >= 2; the
    closed form is checked against the oracle's DPSUB counter first."""
    for n in range(3, 13):
        d = oracle.dpsub(W.star(n, 0))
        assert d.evaluated == 2 * (3 ** (n - 1) - 1)
    g = GOLDEN["star_dpsub_gap"]
    n = g["n"]
    ratio = 2 * (3 ** (n - 1) - 1) / ccp_closed_form("star", n)
    assert math.floor(ratio) == g["ratio"]          # 2805.69
    assert abs(ratio / 2 - g["ratio"]) > 1000        # the ordered reading is ruled out


def test_star_dpsize_gap_printed_ratio():
    """Section 7.2.1: DPSIZE evaluates about 12024x more pairs than MPDP at 20
    relations.  DPSIZE pairs every connected set of size s with every one of
    size i-s; MPDP evaluates the ordered csg-cmp pairs."""
    g = GOLDEN["star_dpsize_gap"]
    n = g["n"]
    # connected sets per size: n singletons, C(n-1, s-1) for s >= 2 (checked below)
    conn = {1: n}
    for s in range(2, n + 1):
        conn[s] = math.comb(n - 1, s - 1)
    q = W.star(12, 0)
    m = oracle.mpdp(q)
    mask = m.has_plan()
    sizes = {}
    for S in range(1, 1 << 12):
        if mask[S]:
            sizes[bin(S).count("1")] = sizes.get(bin(S).count("1"), 0) + 1
    assert sizes == {1: 12, **{s: math.comb(11, s - 1) for s in range(2, 13)}}
    dpsize = sum(conn[s] * conn[i - s] for i in range(2, n + 1) for s in range(1, i))
    ratio = dpsize / (2 * ccp_closed_form("star", n))
    assert math.floor(ratio) == g["ratio"]          # 12024.95
    assert abs(2 * ratio - g["ratio"]) > 1000        # the unordered reading is ruled out


@pytest.mark.parametrize("maker", [lambda s: W.random_tree(10, s), lambda s: W.clique(8, s),
                                   lambda s: W.star(9, s)])
def test_evaluated_equals_ccp_when_blocks_are_cliques(maker):
    """Lemma in Section 3.2.4 (Analysis): if every block is a clique, EvaluatedCounter equals
    CCP-Counter for Alg. 3 (trees: every block is one edge)."""
    q = maker(3)
    m = oracle.mpdp(q, force_general=True)
    assert m.evaluated == m.ccp_ordered


def test_block_enumeration_never_exceeds_dpsub():
    """Section 3.2.4 (Analysis): per set, sum over blocks of 2^(b-1) <= 2^(|S|-1)."""
    for seed in range(4):
        q = W.random_connected(10, seed, 0.25)
        m = oracle.mpdp(q)
        mask = m.has_plan()
        for S in range(1, 1 << q.n):
            if mask[S] and S & (S - 1):
                c = oracle.mpdp_candidates(q, S)
                assert c <= 2 ** bin(S).count("1") - 2
                bl = oracle.blocks(q, S)
                assert c == sum(2 ** bin(b).count("1") - 2 for b in bl)
                # blocks cover S, share at most one vertex, and 1 + sum(b-1) = |S|
                cover = 0
                for b in bl:
                    cover |= b
                assert cover == S
                assert 1 + sum(bin(b).count("1") - 1 for b in bl) == bin(S).count("1")
