"""GPU parity of the large-query heuristics (Section 4) against the oracle.

  * the exact step on units (mpdp_optimize_units, relations with planned
    costs) against the oracle's MPDP with the same base costs, memo and plan
    bit for bit;
  * IDP2 and UnionDP through mpdp_optimize_large against oracle/heuristics.py:
    the same plan node by node and the same cost bits.  UnionDP's parts of at
    most 20 units go through the batched kernel, larger parts and every IDP2
    step through the per-level kernels.
"""
import numpy as np
import pytest

import oracle
from oracle import heuristics as H
from paper_2202_13511_amd import mpdp, workloads as W

pytestmark = pytest.mark.gpu

CMS = [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE]


def bits(x):
    return int(np.float64(x).view(np.uint64))


def with_base_costs(q, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    q.base_cost = 10.0 ** rng.uniform(0.0, 6.0, size=q.n)
    return q


@pytest.mark.parametrize("cm", CMS)
def test_units_exact_step(cm):
    import torch
    qs = [with_base_costs(W.snowflake(14, 1), 1), with_base_costs(W.cycle_chords(3, n=13, chords=4), 2),
          with_base_costs(W.clique(9, 3), 3), with_base_costs(W.random_tree(18, 4), 4),
          with_base_costs(W.chain(2, 5), 5), with_base_costs(W.star(12, 6), 6)]
    for q in qs:
        print(q.name, cm, flush=True)
        ws = mpdp.workspace(q.n, cm, "cuda")
        r = mpdp.mpdp_optimize_units(q, cm, ws)
        m = oracle.mpdp(q, cm)
        assert bits(r.cost) == bits(m.root_cost), q.name
        for nd in r.plan[q.n:]:
            S = nd["relset"]
            assert r.plan[nd["left"]]["relset"] == int(m.left[S]), (q.name, S)
            assert bits(nd["cost"]) == bits(m.cost[S]) and nd["op"] == int(m.op[S]), (q.name, S)
        for v in range(q.n):
            assert bits(r.plan[v]["cost"]) == bits(q.base_cost[v])
        del ws
        torch.cuda.empty_cache()


def same_large(q, cm, method, k):
    r = mpdp.mpdp_optimize_large(q, cm, method, k)
    f = {mpdp.MPDP_LARGE_IDP2: H.idp2, mpdp.MPDP_LARGE_UNIONDP: H.uniondp}[method]
    c, nodes = H.report(q, f(q, k, cm), cm)
    assert bits(r.cost) == bits(c), (q.name, cm, method, k)
    assert len(r.plan) == len(nodes) == 2 * q.n - 1
    for a, b in zip(nodes, r.plan):
        for fld in ("left", "right", "rel", "nrels", "op"):
            assert a[fld] == b[fld], (q.name, cm, method, k, fld)
        assert bits(a["cost"]) == bits(b["cost"]) and bits(a["card"]) == bits(b["card"])
    return r


@pytest.mark.parametrize("cm", CMS)
@pytest.mark.parametrize("method", [mpdp.MPDP_LARGE_IDP2, mpdp.MPDP_LARGE_UNIONDP], ids=["idp2", "uniondp"])
def test_large_parity(cm, method):
    cases = [(W.large_snowflake(60, 11), 5), (W.large_snowflake(100, 12), 10), (W.large_snowflake(150, 13), 15),
             (W.random_connected(40, 14, 0.08), 8), (W.snowflake(25, 15), 25)]
    for q, k in cases:
        print(q.name, cm, method, k, flush=True)
        r = same_large(q, cm, method, k)
        assert r.stats["max_units"] <= k and r.stats["exact_calls"] >= 1


def test_uniondp_parts_beyond_batch_width():
    """k = 22: a part of more than 20 units takes the per-level kernels (a
    22-relation query is one such part); a larger query mixes both paths."""
    q = W.snowflake(22, 21)
    print(q.name, flush=True)
    r = same_large(q, mpdp.MPDP_COST_PGLIKE, mpdp.MPDP_LARGE_UNIONDP, 22)
    assert r.stats["max_units"] == 22
    q = W.large_snowflake(70, 21)
    print(q.name, flush=True)
    same_large(q, mpdp.MPDP_COST_PGLIKE, mpdp.MPDP_LARGE_UNIONDP, 22)


def _hexbits(x):
    return f"{int(np.float64(x).view(np.uint64)):016x}"


def _plan_hash(nodes):
    import hashlib
    lines = [f"{d['left']} {d['right']} {d['rel']} {d['nrels']} {d['op']} {_hexbits(d['cost'])} {_hexbits(d['card'])}"
             for d in nodes]
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def _large_golden():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_large.json")
    return json.load(open(path))["cases"] if os.path.exists(path) else []


def test_large_fullsize_against_stored_oracle():
    """100-1000 relations: plan and cost equal to the oracle's stored results
    (tests/golden/make_large_golden.py)."""
    cases = _large_golden()
    if not cases:
        pytest.skip("no stored oracle results")
    methods = {"goo": mpdp.MPDP_LARGE_GOO, "idp2": mpdp.MPDP_LARGE_IDP2, "uniondp": mpdp.MPDP_LARGE_UNIONDP}
    for g in cases:
        q = W.large_snowflake(g["n"], g["seed"])
        assert q.m == g["m"]
        print(g["name"], g["method"], g["k"], g["cost_model"], flush=True)
        r = mpdp.mpdp_optimize_large(q, g["cost_model"], methods[g["method"]], max(g["k"], 2))
        assert _hexbits(r.cost) == g["cost"], g
        assert _plan_hash(r.plan) == g["plan_sha256"], g


def test_hand_worked_heuristic_cases():
    """The library's IDP2 and UnionDP on the two cases worked by hand in
    tests/test_oracle_heuristics.py: IDP2 from GOO's tree on the five-relation
    chain (k = 3) re-plans {0,1,2} to 0 (1 2) and ends at ((0 (1 2)) 3) 4,
    cost 8472; UnionDP on the six-relation ladder (k = 3) joins its three
    pairs and, through the composite edge of selectivity 0.125, plans
    ((0 1) (2 3)) (4 5), cost 44."""
    from test_oracle_heuristics import _join, _leaf, idp2_chain, union_ladder
    cm = mpdp.MPDP_COST_COUT
    cases = [(idp2_chain(), mpdp.MPDP_LARGE_IDP2, 8472.0,
              _join(_join(_join(_leaf(0), _join(_leaf(1), _leaf(2))), _leaf(3)), _leaf(4))),
             (union_ladder(), mpdp.MPDP_LARGE_UNIONDP, 44.0,
              _join(_join(_join(_leaf(0), _leaf(1)), _join(_leaf(2), _leaf(3))), _join(_leaf(4), _leaf(5))))]
    for q, method, cost, plan in cases:
        r = mpdp.mpdp_optimize_large(q, cm, method, 3)
        assert r.cost == cost, (method, r.cost)
        _, nodes = H.report(q, plan, cm)
        for a, b in zip(r.plan, nodes):
            assert (a["left"], a["right"], a["rel"], a["nrels"], a["op"]) == \
                (b["left"], b["right"], b["rel"], b["nrels"], b["op"]), method


@pytest.mark.parametrize("cm", CMS)
def test_budget_partial_and_generous(cm):
    """A budget that never runs out gives the unbudgeted plan bit for bit; one
    that runs out part way returns MPDP_ETIMEOUT with a complete plan that,
    for IDP2, costs no more than GOO's start (Section 4.1: stop whenever a
    budget is exhausted)."""
    q = W.large_snowflake(300, 1)
    goo_cost = mpdp.mpdp_optimize_large(q, cm, mpdp.MPDP_LARGE_GOO, 2).cost
    for method in (mpdp.MPDP_LARGE_IDP2, mpdp.MPDP_LARGE_UNIONDP):
        print(q.name, cm, method, flush=True)
        full = mpdp.mpdp_optimize_large(q, cm, method, 15)
        r = mpdp.mpdp_optimize_large(q, cm, method, 15, budget_ms=1e6)
        assert not r.stats["timed_out"] and bits(r.cost) == bits(full.cost)
        assert r.plan == full.plan
        r = mpdp.mpdp_optimize_large(q, cm, method, 15, budget_ms=max(0.3 * full.stats["ms_total"], 0.05))
        assert r.stats["timed_out"], (q.name, method)
        assert r.plan[-1]["nrels"] == q.n and len(r.plan) == 2 * q.n - 1
        if method == mpdp.MPDP_LARGE_IDP2:
            assert r.cost <= goo_cost
