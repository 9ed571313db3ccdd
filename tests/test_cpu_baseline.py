"""The all-cores CPU MPDP (mpdp_optimize_cpu, host threads, no GPU) against
the oracle: plan node by node, every join's cost bit for bit, and the
counters, on tree, cyclic and dense graphs, both cost models, one and
several threads."""
import numpy as np
import pytest

import oracle
from paper_2202_13511_amd import mpdp, workloads as W

CMS = [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE]


def queries():
    return [W.star(12, 1), W.snowflake(16, 2), W.chain(14, 3), W.cycle_chords(4, n=14, chords=4),
            W.clique(10, 5), W.random_connected(13, 6, 0.3), W.all_equal_clique(8), W.random_tree(15, 7)]


@pytest.mark.parametrize("cm", CMS)
@pytest.mark.parametrize("threads", [1, 4])
def test_cpu_mpdp_matches_oracle(cm, threads):
    for q in queries():
        r = mpdp.mpdp_optimize_cpu(q, cm, threads)
        m = oracle.mpdp(q, cm)
        assert np.float64(r.cost).view(np.uint64) == np.float64(m.root_cost).view(np.uint64), q.name
        for nd in r.plan[q.n:]:
            S = nd["relset"]
            assert r.plan[nd["left"]]["relset"] == int(m.left[S]), (q.name, S)
            assert np.float64(nd["cost"]).view(np.uint64) == m.cost[S].view(np.uint64)
            assert nd["op"] == int(m.op[S])
        assert r.stats["connected_sets"] == m.connected_sets, q.name
        assert r.stats["ccp_pairs"] * 2 == m.ccp_ordered, q.name
        assert r.stats["evaluated_pairs"] == m.evaluated, q.name


def test_cpu_mpdp_validation():
    with pytest.raises(mpdp.MpdpError) as e:
        mpdp.mpdp_optimize_cpu(W.chain(29, 0))
    assert e.value.status == mpdp.MPDP_ETOOLARGE
    disc = W.Query(4, np.array([[0, 1], [2, 3]], np.uint32), np.full(4, 10.0), np.full(2, 0.5))
    with pytest.raises(mpdp.MpdpError) as e:
        mpdp.mpdp_optimize_cpu(disc)
    assert e.value.status == mpdp.MPDP_ENOTCONNECTED
