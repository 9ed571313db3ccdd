#!/usr/bin/env python3
"""Write tests/golden/oracle_fullsize.json from the CPU oracle only.

For every full-size workload query it stores what the GPU must reproduce bit
for bit: the root cost, the plan (relation set, left input set and operator
of every join node), the counters, and 32 memo entries of connected sets
drawn with a fixed seed.  Nothing here calls the HIP library.

Workloads (generators in paper_2202_13511_amd.workloads):
  star12      hub + 11 leaves, seeds 0..63, C_out
  star25      hub + 24 leaves, seeds 0..15, C_out and PG-like
  snowflake25 depth 3, fanout U{2..4}, seeds 0..63, C_out and PG-like
  clique18    seeds 0..31, C_out and PG-like
  cycle       ring of U{20..30} + U{5..15} chords, seeds 0..31, C_out; and
              the seeds of 20-23 relations also under PG-like (its Alg. 3
              path through the heavy-set kernel on sparse blocks)

Every query is solved whole.  For the cyclic queries of 27 or more
relations (whose whole solution takes the oracle from minutes to hours) the
file also holds sub-query checks ("cycle_sub"): 4 connected sets of 20-24
relations and 12 of 3-16, grown by a seeded random walk, each solved by the
oracle on its induced sub-query (a set's memo entry depends only on the
relations and edges inside it, so the whole query's entry must equal the
sub-query's root).  The file is updated in place: queries already
stored are kept (unless --force) and the file is rewritten after every
query solved, so an interrupted run resumes where it stopped.  Queries of
up to 25 relations run in a pool of single-threaded workers; larger ones run
one at a time with the oracle's level split over --threads threads (a
30-relation memo takes 22.5 GB of host memory).

Usage: python tests/golden/make_oracle_golden.py [--jobs 8] [--threads 8] [--force]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_fullsize.json")
SAMPLES = 32
SUB_MIN_N = 27


def spec_list():
    specs = [("star", 12, s, 0) for s in range(64)]
    specs += [("star", 25, s, cm) for cm in (0, 1) for s in range(16)]
    specs += [("snowflake", 25, s, cm) for cm in (0, 1) for s in range(64)]
    specs += [("clique", 18, s, cm) for cm in (0, 1) for s in range(32)]
    specs += [("cycle_chords", None, s, 0) for s in range(32)]
    specs += [("cycle_chords", None, s, 1) for s in range(32) if make_query("cycle_chords", None, s).n <= 23]
    specs += [("cycle_sub", None, s, 0) for s in range(32) if make_query("cycle_chords", None, s).n >= SUB_MIN_N]
    return specs


def make_query(kind, n, seed):
    from paper_2202_13511_amd import workloads as W
    if kind == "star":
        return W.star(n, seed)
    if kind == "snowflake":
        return W.snowflake(n, seed)
    if kind == "clique":
        return W.clique(n, seed)
    if kind in ("cycle_chords", "cycle_sub"):
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


def sub_checks(q, seed, cm, threads):
    """Connected sets of q solved by the oracle on their induced sub-queries
    (relabelled in increasing order, which leaves every value unchanged)."""
    import oracle
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    sizes = [int(rng.integers(20, 25)) for _ in range(4)] + [int(rng.integers(3, 17)) for _ in range(12)]
    samples, seen = [], set()
    for size in sizes:
        while True:
            S = random_connected_set(q, rng, size)
            if S not in seen:
                break
        seen.add(S)
        sub, rel = oracle.induced(q, S)
        m = oracle.mpdp(sub, cm, threads=threads if size > 18 else 1)
        samples.append([int(S), hexbits(m.root_cost), hexbits(m.card[m.full]),
                        oracle.expand(rel, int(m.left[m.full])), int(m.op[m.full])])
    return {"kind": "cycle_sub", "n": q.n, "seed": seed, "cost_model": cm, "name": q.name, "m": q.m,
            "sampled_only": True, "samples": samples}


def key(kind, seed, cm):
    return f"{kind}/{seed}/{cm}"


def one(spec, threads=1):
    import oracle
    kind, n, seed, cm = spec
    if kind == "cycle_sub":
        return sub_checks(make_query("cycle_chords", n, seed), seed, cm, threads)
    q = make_query(kind, n, seed)
    m = oracle.mpdp(q, cm, threads=threads)
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
    out = {
        "kind": kind, "n": q.n, "seed": seed, "cost_model": cm, "name": q.name, "m": q.m,
        "root_cost": hexbits(m.root_cost), "joins": joins,
        "connected_sets": m.connected_sets, "ccp_pairs": m.ccp_ordered // 2, "evaluated_pairs": evaluated,
        "samples": samples,
    }
    del m, mask, conn  # a 30-relation memo is 22.5 GB: free it before the next query
    return out


ABOUT = ("Expected results of the CPU oracle (oracle.mpdp) on the full-size workloads; written by "
         "tests/golden/make_oracle_golden.py, which calls only oracle/ and the input generators. "
         "Costs and cards are IEEE binary64 bit patterns in hex; joins are [relation set, left input "
         "set, operator] in plan post-order; samples are [set, cost, card, left, op].")


def save(done, order):
    """Write the stored queries in spec order (atomic replace)."""
    results = [done[k] for k in order if k in done]
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"_about": ABOUT, "queries": results}, f, separators=(",", ":"))
        f.write("\n")
    os.replace(tmp, OUT)
    return len(results)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--force", action="store_true", help="solve every query again")
    specs = spec_list()
    order = [key(k, s, cm) for k, _, s, cm in specs]
    done = {}
    ap.add_argument("--only", default="", help="solve only specs of this kind")
    args = ap.parse_args()
    if os.path.exists(OUT) and not args.force:
        for g in json.load(open(OUT))["queries"]:
            if g["kind"] == "cycle_sub" or not g.get("sampled_only"):
                done[key(g["kind"], g["seed"], g["cost_model"])] = g
    todo = [sp for sp in specs if key(sp[0], sp[2], sp[3]) not in done and (not args.only or sp[0] == args.only)]
    small = [sp for sp in todo if make_query(sp[0], sp[1], sp[2]).n <= 25]
    # sub-query checks first, then whole queries by size
    large = sorted((sp for sp in todo if sp not in small),
                   key=lambda sp: (sp[0] != "cycle_sub", make_query(sp[0], sp[1], sp[2]).n))
    with ProcessPoolExecutor(args.jobs) as ex:
        for r in ex.map(one, small):
            done[key(r["kind"], r["seed"], r["cost_model"])] = r
    if small:
        print(f"stored {save(done, order)} queries", flush=True)
    for sp in large:
        t = time.perf_counter()
        r = one(sp, args.threads)
        done[key(r["kind"], r["seed"], r["cost_model"])] = r
        stored = save(done, order)
        print(f"{r['name']} cm={r['cost_model']}: {time.perf_counter() - t:.0f} s, {stored} stored", flush=True)
    print(f"{save(done, order)} queries in {OUT}")


if __name__ == "__main__":
    main()
