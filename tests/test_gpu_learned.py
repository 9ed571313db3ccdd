"""GPU parity of the learned UnionDP pipeline against the oracle.

  * training examples (features of every candidate union of every pass of
    the learned partition phase driven by the teacher, labels from an
    optimal plan) bit for bit against oracle/heuristics.py's, for plans of
    20-26 relations;
  * the learned union order end to end: with weights whose arithmetic is
    exact in float32 (entries 0 or +-1, at most three terms per unit and
    bfloat16 inputs), the device's logits equal the oracle's, so the plans
    must be equal node for node and the cost bit for bit.
"""
import numpy as np
import pytest

import oracle
from oracle import heuristics as H
from oracle import mlp
from paper_2202_13511_amd import mpdp, workloads as W

pytestmark = pytest.mark.gpu


def bits(x):
    return int(np.float64(x).view(np.uint64))


def optimal_sets(q, cm):
    m = oracle.mpdp(q, cm)
    plan = oracle.plan_from_memo(m)
    return {nd["relset"] for nd in plan}


@pytest.mark.parametrize("cm", [0, 1])
def test_examples_match_oracle(cm):
    for n, seed, k in ((20, 1, 4), (22, 2, 6), (26, 3, 8)):
        q = W.large_snowflake(n, seed)
        print(q.name, cm, k, flush=True)
        sets = optimal_sets(q, cm)
        X, y = mpdp.mpdp_large_examples(q, cm, k, sets)
        ex = []
        H.uniondp(q, k, cm, examples=ex, plan_sets=sets, teacher=True)
        Xo = np.concatenate([e[0] for e in ex])
        yo = np.concatenate([e[1] for e in ex])
        assert X.shape == Xo.shape and np.array_equal(X, Xo), q.name
        assert np.array_equal(y, yo.astype(np.float32)), q.name
        assert 0 < y.sum() < len(y)


def exact_weights(seed):
    """Sparse +-1 weights: every float32 sum of the network is exact."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1 = np.zeros((mlp.IN, mlp.HID), np.float32)
    for h in range(mlp.HID):
        for f in rng.choice(19, 3, replace=False):
            w1[f, h] = rng.choice([-1.0, 1.0])
    w2 = np.zeros((mlp.HID, mlp.HID), np.float32)
    for o in range(mlp.HID):
        for i in rng.choice(mlp.HID, 2, replace=False):
            w2[i, o] = rng.choice([-1.0, 1.0])
    w3 = np.zeros(mlp.HID, np.float32)
    w3[rng.choice(mlp.HID, 4, replace=False)] = rng.choice([-1.0, 1.0], 4)
    z = np.zeros(mlp.HID, np.float32)
    return dict(w1=w1, b1=z, w2=w2, b2=z.copy(), w3=w3, b3=np.zeros(1, np.float32))


@pytest.mark.parametrize("cm", [0, 1])
def test_learned_order_parity(cm):
    for n, seed, k, wseed in ((60, 5, 6, 1), (150, 6, 10, 2), (40, 7, 15, 3)):
        q = W.large_snowflake(n, seed)
        print(q.name, cm, k, flush=True)
        w = exact_weights(wseed)
        block = mpdp.scorer_params()
        mpdp.scorer_load(block, w)
        r = mpdp.mpdp_optimize_large(q, cm, mpdp.MPDP_LARGE_UNIONDP_LEARNED, k, scorer=block)
        plan = H.uniondp(q, k, cm, scorer=lambda X: mlp.forward(w, X)[0])
        c, nodes = H.report(q, plan, cm)
        assert bits(r.cost) == bits(c), q.name
        for a, b in zip(nodes, r.plan):
            for fld in ("left", "right", "rel", "nrels", "op"):
                assert a[fld] == b[fld], (q.name, fld)


def test_trained_scorer_against_plain_uniondp():
    """Train the scorer on the GPU (teacher round, then DAgger rounds on the
    network's own unions; plans of 20-26 relations from the exact DP) and
    measure what it gains over plain UnionDP on held-out queries, with the
    exact DP as the reference: geometric-mean ratio to the optimum at k = 15
    under C_out.  The run is deterministic (fixed draws, no atomics in the
    gradient sums), so the comparison is stable."""
    from paper_2202_13511_amd import scorer
    block, log = scorer.train(mpdp.MPDP_COST_COUT, seed=1, queries=300, rounds=4, steps=3000)
    print("train", log, flush=True)
    assert log.loss[-1] < 0.5 * 0.693  # well below the loss of a constant guess
    held = scorer.training_queries(40, 99)
    plain, learned = scorer.compare_small(block, mpdp.MPDP_COST_COUT, held, 15)
    gp, gl = float(np.exp(np.mean(np.log(plain)))), float(np.exp(np.mean(np.log(learned))))
    print(f"k=15 geometric mean ratio to optimum: plain {gp:.3f} learned {gl:.3f}; "
          f"learned better on {np.mean(learned < plain):.2f}, worse on {np.mean(learned > plain):.2f}", flush=True)
    assert np.all(learned >= 1.0 - 1e-12) and np.all(plain >= 1.0 - 1e-12)
    # what the network gains: a lower geometric-mean ratio to the optimum
    # than the paper's partition order at the same k (9.57 against 10.40
    # when this was written)
    assert gl < gp, (gl, gp)
