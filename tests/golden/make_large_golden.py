"""Write tests/golden/oracle_large.json from the CPU oracle alone.

Large-query workload (100-1000 relations, snowflake of depth <= 4 plus random
cross edges): GOO, IDP2 and UnionDP planned by oracle/heuristics.py, the
exact step being the oracle's MPDP.  Each entry stores the re-costed plan
cost (IEEE bit pattern, hex) and a SHA-256 of the flat plan (one line per
node: left right rel nrels op cost-hex card-hex).  Slow (minutes: GOO and
IDP2 in plain Python scan every pair and subtree); run it from the
repository root:

    python tests/golden/make_large_golden.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import heuristics as H  # noqa: E402
from paper_2202_13511_amd import workloads as W  # noqa: E402

CASES = [  # n, seed, cost model (0 C_out, 1 PG-like), method, k
    (100, 0, 1, "uniondp", 15), (100, 0, 1, "idp2", 15), (100, 0, 1, "goo", 0),
    (100, 0, 0, "uniondp", 15), (100, 0, 0, "idp2", 15), (100, 0, 1, "idp2", 25),
    (300, 0, 1, "uniondp", 15), (300, 0, 1, "idp2", 15), (300, 0, 1, "goo", 0),
    (1000, 0, 1, "uniondp", 15), (1000, 0, 1, "uniondp", 25), (1000, 0, 1, "goo", 0),
]


def hexbits(x):
    return f"{int(np.float64(x).view(np.uint64)):016x}"


def plan_hash(nodes):
    lines = [f"{d['left']} {d['right']} {d['rel']} {d['nrels']} {d['op']} {hexbits(d['cost'])} {hexbits(d['card'])}"
             for d in nodes]
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def main():
    out = []
    for n, seed, cm, method, k in CASES:
        q = W.large_snowflake(n, seed)
        t = time.time()
        if method == "goo":
            plan = H.goo(q, cm)
        elif method == "idp2":
            plan = H.idp2(q, k, cm)
        else:
            plan = H.uniondp(q, k, cm)
        cost, nodes = H.report(q, plan, cm)
        out.append(dict(name=q.name, n=n, seed=seed, m=q.m, cost_model=cm, method=method, k=k,
                        cost=hexbits(cost), plan_sha256=plan_hash(nodes)))
        print(f"{q.name} cm={cm} {method}{k or ''}: cost {cost:.6g} ({time.time() - t:.1f} s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_large.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_large_golden.py", "cases": out}, f, indent=1)


if __name__ == "__main__":
    main()
