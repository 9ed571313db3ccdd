"""Host logic of the large-query entry point that needs no GPU: input
validation and GOO (which never calls the exact step), against the oracle."""
import numpy as np
import pytest

from oracle import heuristics as H
from paper_2202_13511_amd import mpdp, workloads as W

CMS = [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE]


def bits(x):
    return int(np.float64(x).view(np.uint64))


@pytest.mark.parametrize("cm", CMS)
def test_goo_matches_oracle(cm):
    for q in [W.snowflake(14, 3), W.cycle_chords(2, n=12, chords=3), W.large_snowflake(100, 1),
              W.large_snowflake(150, 2), W.random_connected(30, 1, 0.1), W.star(9, 4)]:
        r = mpdp.mpdp_optimize_large(q, cm, mpdp.MPDP_LARGE_GOO, 2)
        c, nodes = H.report(q, H.goo(q, cm), cm)
        assert bits(r.cost) == bits(c), q.name
        for a, b in zip(nodes, r.plan):
            for f in ("left", "right", "rel", "nrels", "op"):
                assert a[f] == b[f], (q.name, f)
            assert bits(a["cost"]) == bits(b["cost"]) and bits(a["card"]) == bits(b["card"])


def test_large_validation():
    def status(q, method=mpdp.MPDP_LARGE_UNIONDP, k=10):
        try:
            mpdp.mpdp_optimize_large(q, 0, method, k)
        except mpdp.MpdpError as e:
            return e.status
        return mpdp.MPDP_OK

    good = W.chain(5, 0)
    assert status(good, k=1) == mpdp.MPDP_EINVAL
    assert status(good, k=26) == mpdp.MPDP_EINVAL
    assert status(good, method=7) == mpdp.MPDP_EINVAL
    assert status(W.chain(4100, 1)) == mpdp.MPDP_ETOOLARGE
    bad = W.chain(6, 2)
    bad.edges = np.vstack([bad.edges, bad.edges[:1, ::-1]])  # the same predicate twice
    bad.sel = np.append(bad.sel, 0.5)
    assert status(bad) == mpdp.MPDP_EINVAL
    disc = W.Query(4, np.array([[0, 1], [2, 3]], np.uint32), np.full(4, 10.0), np.full(2, 0.5))
    assert status(disc) == mpdp.MPDP_ENOTCONNECTED
    one = W.Query(1, np.zeros((0, 2), np.uint32), np.array([50.0]), np.zeros(0))
    r = mpdp.mpdp_optimize_large(one, mpdp.MPDP_COST_PGLIKE, mpdp.MPDP_LARGE_GOO, 2)
    assert r.cost == 0.5 and r.plan[0]["rel"] == 0


@pytest.mark.parametrize("cm", CMS)
def test_budget_exhausted_before_any_exact_step(cm):
    """Section 4.1's budget: a budget that is over before the first exact
    sub-problem leaves IDP2 with its GOO start, and UnionDP joins its units
    (still single relations) by GOO; both report MPDP_ETIMEOUT with the plan,
    and no HIP call is made."""
    for q in [W.large_snowflake(100, 1), W.snowflake(14, 3), W.cycle_chords(2, n=12, chords=3)]:
        c, nodes = H.report(q, H.goo(q, cm), cm)
        for method in (mpdp.MPDP_LARGE_IDP2, mpdp.MPDP_LARGE_UNIONDP):
            r = mpdp.mpdp_optimize_large(q, cm, method, 10, budget_ms=1e-9)
            assert r.stats["timed_out"], q.name
            assert bits(r.cost) == bits(c), (q.name, method)
            for a, b in zip(nodes, r.plan):
                for f in ("left", "right", "rel", "nrels", "op"):
                    assert a[f] == b[f], (q.name, method, f)
        # GOO ignores the budget
        r = mpdp.mpdp_optimize_large(q, cm, mpdp.MPDP_LARGE_GOO, 2, budget_ms=1e-9)
        assert not r.stats["timed_out"] and bits(r.cost) == bits(c)


def test_budget_validation():
    q = W.chain(8, 0)
    for b in (-1.0, float("nan"), float("inf")):
        with pytest.raises(mpdp.MpdpError) as e:
            mpdp.mpdp_optimize_large(q, 0, mpdp.MPDP_LARGE_IDP2, 5, budget_ms=b)
        assert e.value.status == mpdp.MPDP_EINVAL
