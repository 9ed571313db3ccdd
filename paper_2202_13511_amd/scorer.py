"""Training and evaluation driver of the learned UnionDP scorer.

Every computation runs in the library: the exact plans that give the labels
(mpdp_optimize on the GPU), the candidate unions and their features
(mpdp_large_examples), the network's forward and backward passes and the
Adam steps (mpdp_scorer_* on the matrix cores), and the heuristics being
compared (mpdp_optimize_large).  This module only draws the training
queries and the minibatches and loops.

Training is imitation with aggregation (DAgger): the first round collects
the unions the teacher (the optimal plan's nodes) would make, later rounds
the unions the current network makes, all labelled by the optimal plan; the
network is retrained on everything collected so far.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import mpdp
from . import workloads as W


def training_queries(count: int, seed: int, n_range=(20, 26)):
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(n_range[0], n_range[1] + 1, count)
    return [W.large_snowflake(int(n), int(seed) * 100003 + i) for i, n in enumerate(ns)]


def optimal_sets(q, cm: int):
    """Relation sets of the nodes of the exact DP's plan (and its cost)."""
    r = mpdp.mpdp_optimize(q, cm)
    return {nd["relset"] for nd in r.plan}, r.cost


def init_weights(seed: int) -> dict:
    """He-uniform weights, zero biases (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    IN, HID = mpdp.SCORER_IN, mpdp.SCORER_HIDDEN

    def he(fan_in, shape):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=shape).astype(np.float32)

    return dict(w1=he(IN, (IN, HID)), b1=np.zeros(HID, np.float32), w2=he(HID, (HID, HID)),
                b2=np.zeros(HID, np.float32), w3=he(HID, (HID,)), b3=np.zeros(1, np.float32))


@dataclass
class TrainLog:
    examples: list = field(default_factory=list)   # rows per round
    positives: list = field(default_factory=list)  # share of label 1 per round
    loss: list = field(default_factory=list)       # last minibatch loss per round


def train(cm: int, seed: int = 0, queries: int = 160, ks=(5, 8, 12), rounds: int = 3, steps: int = 2000,
          batch: int = 512, lr: float = 1e-3):
    """Train a scorer for cost model `cm`; returns (device parameter block, TrainLog)."""
    import torch
    qs = training_queries(queries, seed)
    sets = [optimal_sets(q, cm)[0] for q in qs]
    block = mpdp.scorer_params()
    mpdp.scorer_load(block, init_weights(seed))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    work = mpdp.scorer_work(batch)
    Xs, ys = [], []
    log = TrainLog()
    step = 0
    for rnd in range(rounds):
        policy = None if rnd == 0 else block  # teacher first, then the network itself
        for q, S in zip(qs, sets):
            for k in ks:
                X, y = mpdp.mpdp_large_examples(q, cm, k, S, scorer=policy)
                Xs.append(X)
                ys.append(y)
        X = np.concatenate(Xs)
        y = np.concatenate(ys)
        Xd = torch.from_numpy(X.view(np.int16)).to(block.device)
        yd = torch.from_numpy(y).to(block.device)
        loss = 0.0
        for it in range(steps):
            idx = torch.from_numpy(rng.integers(0, len(y), batch)).to(block.device)
            step += 1
            loss = mpdp.scorer_train_step(block, Xd[idx], yd[idx], lr, step, work=work,
                                          want_loss=(it == steps - 1))
        log.examples.append(int(len(y)))
        log.positives.append(float(y.mean()))
        log.loss.append(float(loss))
    return block, log


def compare_small(block, cm: int, queries, k: int):
    """Plan-cost ratios to the exact optimum of plain and learned UnionDP."""
    plain, learned = [], []
    for q in queries:
        _, best = optimal_sets(q, cm)
        plain.append(mpdp.mpdp_optimize_large(q, cm, mpdp.MPDP_LARGE_UNIONDP, k).cost / best)
        learned.append(mpdp.mpdp_optimize_large(q, cm, mpdp.MPDP_LARGE_UNIONDP_LEARNED, k, scorer=block).cost / best)
    return np.array(plain), np.array(learned)
