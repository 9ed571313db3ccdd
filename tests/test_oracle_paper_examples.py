"""The paper's worked examples (tests/golden/paper_examples.json) against the oracle."""
import json
import os

import numpy as np

import oracle
from paper_2202_13511_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def bm(labels):
    s = 0
    for v in labels:
        s |= 1 << (v - 1)
    return s


def nine():
    g = GOLDEN["nine_relation_example"]
    e = np.array([[a - 1, b - 1] for a, b in g["edges"]], np.uint32)
    return g, W.from_edges(9, e, 0, "paper-9")


def connected(q, S):
    return S != 0 and oracle.grow(q, S & -S, S) == S


def test_nine_relation_blocks_and_cut_vertices():
    g, q = nine()
    full = (1 << 9) - 1
    assert oracle.blocks(q, full) == sorted(bm(b) for b in g["blocks"])
    cuts = [v + 1 for v in range(9) if not connected(q, full & ~(1 << v))]
    assert cuts == g["cut_vertices"]
    # block-cut tree: consecutive blocks share exactly the cut vertex between them
    chain = g["block_cut_tree_chain"]
    for i in range(0, len(chain) - 2, 2):
        assert bm(chain[i]) & bm(chain[i + 2]) == 1 << (chain[i + 1] - 1)


def test_nine_relation_grow_example():
    g, q = nine()
    gr = g["grow"]
    assert oracle.grow(q, bm(gr["source"]), bm(gr["restriction"])) == bm(gr["result"])


def test_nine_relation_512_vs_32():
    g, q = nine()
    full = (1 << 9) - 1
    assert 2 ** 9 == g["dpsub_evaluations_full_set"]
    assert oracle.mpdp_candidates(q, full) == g["mpdp_evaluations_full_set"]


def test_nine_relation_removed_edge_is_not_a_pair():
    """Removing edge (1,4) of the cyclic example does not split the graph."""
    g, q = nine()
    a, b = g["removed_edge_not_a_pair"]
    keep = [(u, v) for u, v in q.edges.tolist() if {u, v} != {a - 1, b - 1}]
    q2 = W.from_edges(9, keep, 0)
    assert connected(q2, (1 << 9) - 1)


def test_figure1_join_pairs():
    g = GOLDEN["fig1_tpch_chain"]
    idx = {r: i for i, r in enumerate(g["relations"])}
    e = [(idx[a], idx[b]) for a, b in g["predicates"]]
    q = W.from_edges(4, e, 0, "fig1")

    def is_ccp(A, B):
        return (A and B and not A & B and connected(q, A) and connected(q, B)
                and oracle.grow(q, A, A | B) == A | B)

    for a, b in g["invalid_pairs"]:
        assert not is_ccp(1 << idx[a], 1 << idx[b])
    for a, b in g["valid_pairs"]:
        assert is_ccp(1 << idx[a], 1 << idx[b])
    assert oracle.count_ccp(q) == 10  # a 4-chain: (4^3 - 4) / 6
