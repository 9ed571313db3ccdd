#!/usr/bin/env python3
"""Write tests/golden/oracle_fullsize.json from the CPU oracle only.

For every full-size workload query it stores what the GPU must reproduce bit
for bit: the root cost, the plan (relation set, left input set and operator
of every join node), the counters, and 32 memo entries of connected sets
drawn with a fixed seed.  Nothing here calls the HIP library.

Workloads (generators in paper_2202_13511_amd.workloads):
  star12      hub + 11 leaves, seeds 0..63, C_out
  star25      hub + 24 leaves, seeds 0..15, C_out and PG-like
  snowflake25 depth 3, fanout U{2..4}, seeds 0..63 C_out, 0..15 PG-like
  clique18    seeds 0..31, C_out
  cycle       ring of U{20..30} + U{5..15} chords, seeds 0..31, C_out: whole
              query when n <= 22; for larger n (beyond the oracle's time
              budget for a whole query) 16 connected sets per query drawn by
              a seeded random walk, each solved by the oracle on its induced
              sub-query (relabelled in increasing order, which leaves every
              memo value unchanged)

Usage: python tests/golden/make_oracle_golden.py [--jobs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_fullsize.json")
SAMPLES = 32


def spec_list():
    specs = [("star", 12, s, 0) for s in range(64)]
    specs += [("star", 25, s, cm) for cm in (0, 1) for s in range(16)]
    specs += [("snowflake", 25, s, 0) for s in range(64)]
    specs += [("snowflake", 25, s, 1) for s in range(16)]
    specs += [("clique", 18, s, 0) for s in range(32)]
    specs += [("cycle_chords", None, s, 0) for s in range(32)]
    return specs


def make_query(kind, n, seed):
    from paper_2202_13511_amd import workloads as W
    if kind == "star":
        return W.star(n, seed)
    if kind == "snowflake":
        return W.snowflake(n, seed)
    if kind == "clique":
        return W.clique(n, seed)
    if kind == "cycle_chords":
        return W.cycle_chords(seed)
    raise ValueError(kind)


def hexbits(x) -> str:
    return f"{int(np.float64(x).view(np.uint64)):016x}"


def random_connected_set(q, rng, size):
    adj = q.adjacency()
    S = 1 << int(rng.integers(0, q.n))
    while bin(S).count("1") < size:
        frontier = 0
        for v in range(q.n):
            if S >> v & 1:
                frontier |= adj[v]
        frontier &= ~S
        cand = [v for v in range(q.n) if frontier >> v & 1]
        S |= 1 << cand[int(rng.integers(0, len(cand)))]
    return S


def sampled(q, kind, seed, cm):
    import oracle
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    samples = []
    seen = set()
    while len(samples) < 16:
        S = random_connected_set(q, rng, int(rng.integers(3, 17)))
        if S in seen:
            continue
        seen.add(S)
        sub, rel = oracle.induced(q, S)
        m = oracle.mpdp(sub, cm)
        samples.append([int(S), hexbits(m.root_cost), hexbits(m.card[m.full]),
                        oracle.expand(rel, int(m.left[m.full])), int(m.op[m.full])])
    return {"kind": kind, "n": q.n, "seed": seed, "cost_model": cm, "name": q.name, "m": q.m,
            "sampled_only": True, "samples": samples}


def one(spec):
    import oracle
    kind, n, seed, cm = spec
    q = make_query(kind, n, seed)
    if kind == "cycle_chords" and q.n > 22:
        return sampled(q, kind, seed, cm)
    m = oracle.mpdp(q, cm)
    tree = q.m == q.n - 1
    evaluated = m.evaluated if not tree else m.ccp_ordered
    plan = oracle.plan_from_memo(m)
    joins = [[nd["relset"], plan[nd["left"]]["relset"], nd["op"]] for nd in plan[q.n:]]
    mask = m.has_plan()
    conn = np.nonzero(mask)[0]
    conn = conn[conn & (conn - 1) != 0]  # at least two relations
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    pick = np.sort(rng.choice(conn, size=min(SAMPLES, conn.size), replace=False))
    samples = [[int(S), hexbits(m.cost[S]), hexbits(m.card[S]), int(m.left[S]), int(m.op[S])] for S in pick]
    return {
        "kind": kind, "n": q.n, "seed": seed, "cost_model": cm, "name": q.name, "m": q.m,
        "root_cost": hexbits(m.root_cost), "joins": joins,
        "connected_sets": m.connected_sets, "ccp_pairs": m.ccp_ordered // 2, "evaluated_pairs": evaluated,
        "samples": samples,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    specs = spec_list()
    with ProcessPoolExecutor(args.jobs) as ex:
        results = [r for r in ex.map(one, specs) if r is not None]
    doc = {
        "_about": "Expected results of the CPU oracle (oracle.mpdp) on the full-size workloads; written by "
                  "tests/golden/make_oracle_golden.py, which calls only oracle/ and the input generators. "
                  "Costs and cards are IEEE binary64 bit patterns in hex; joins are [relation set, left input "
                  "set, operator] in plan post-order; samples are [set, cost, card, left, op].",
        "queries": results,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
        f.write("\n")
    print(f"wrote {len(results)} queries to {OUT}")


if __name__ == "__main__":
    main()
