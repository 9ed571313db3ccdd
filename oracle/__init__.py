"""CPU oracle for the MPDP join-order dynamic program (arXiv 2202.13511).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path (the HIP library and
its Python binding) never imports this package, and this package never
imports the product path; both read the same seeded inputs from
``paper_2202_13511_amd.workloads``.

Contents
  mpdp_oracle.c   DPSUB (Alg. 1), MPDP (Alg. 2 on trees, Alg. 3 with
                  Hopcroft-Tarjan blocks), DPccp csg-cmp enumeration and a
                  level-bucketed DPccp DP, card(S), grow, blocks.
  bruteforce.py   every cross-product-free bushy tree, for n <= 7.
  special.py      textbook special cases: the chain interval DP and the
                  optimal star order under C_out.

The shared definitions (card(S), the two cost models, the plan key) are
written out in the header comment of mpdp_oracle.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpdp_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "liboracle.so")

COST_COUT = 0
COST_PGLIKE = 1
OP_SCAN, OP_HASH, OP_NESTLOOP, OP_JOIN = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        f64p = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i = ctypes.c_int
        memo_sig = [i, i, u32p, f64p, f64p, i]
        out_sig = [f64p, f64p, u32p, u8p, u64p]
        L.oracle_dpsub.argtypes = memo_sig + out_sig
        L.oracle_dpsub.restype = i
        L.oracle_mpdp.argtypes = memo_sig + [i] + out_sig
        L.oracle_mpdp.restype = i
        L.oracle_mpdp_threads.argtypes = memo_sig + [i, i] + out_sig
        L.oracle_mpdp_threads.restype = i
        L.oracle_mpdp_bc.argtypes = memo_sig + [f64p] + out_sig
        L.oracle_mpdp_bc.restype = i
        L.oracle_dpccp.argtypes = memo_sig + out_sig
        L.oracle_dpccp.restype = i
        L.oracle_count_ccp.argtypes = [i, i, u32p]
        L.oracle_count_ccp.restype = ctypes.c_uint64
        L.oracle_card.argtypes = [i, i, u32p, f64p, f64p, ctypes.c_uint32, f64p]
        L.oracle_card.restype = i
        L.oracle_grow.argtypes = [i, i, u32p, ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_grow.restype = ctypes.c_uint32
        L.oracle_blocks.argtypes = [i, i, u32p, ctypes.c_uint32, u32p]
        L.oracle_blocks.restype = i
        L.oracle_mpdp_candidates.argtypes = [i, i, u32p, ctypes.c_uint32]
        L.oracle_mpdp_candidates.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _inputs(q):
    e = np.ascontiguousarray(q.edges, dtype=np.uint32).reshape(-1)
    c = np.ascontiguousarray(q.card, dtype=np.float64)
    s = np.ascontiguousarray(q.sel, dtype=np.float64)
    return e, c, s


@dataclass
class Memo:
    """Dense memo indexed by the relation-set bitmap (size 2^n)."""
    n: int
    cost: np.ndarray
    card: np.ndarray
    left: np.ndarray
    op: np.ndarray
    evaluated: int
    ccp_ordered: int
    connected_sets: int

    @property
    def full(self) -> int:
        return (1 << self.n) - 1

    @property
    def root_cost(self) -> float:
        return float(self.cost[self.full])

    def has_plan(self) -> np.ndarray:
        """Boolean mask of sets with a plan (connected sets incl. singletons)."""
        m = self.left != 0
        for v in range(self.n):
            m[1 << v] = True
        return m


def _run(fn, q, cost_model, *extra):
    n = q.n
    N = 1 << n
    cost = np.empty(N, np.float64)
    card = np.empty(N, np.float64)
    left = np.empty(N, np.uint32)
    op = np.empty(N, np.uint8)
    cnt = np.zeros(3, np.uint64)
    e, c, s = _inputs(q)
    rc = fn(n, q.m, _p(e, ctypes.c_uint32), _p(c, ctypes.c_double), _p(s, ctypes.c_double),
            int(cost_model), *extra, _p(cost, ctypes.c_double), _p(card, ctypes.c_double),
            _p(left, ctypes.c_uint32), _p(op, ctypes.c_uint8), _p(cnt, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"oracle rejected the query (rc={rc})")
    return Memo(n, cost, card, left, op, int(cnt[0]), int(cnt[1]), int(cnt[2]))


def dpsub(q, cost_model=COST_COUT) -> Memo:
    """Generic DPSUB, Alg. 1 (n <= 20)."""
    return _run(lib().oracle_dpsub, q, cost_model)


def mpdp(q, cost_model=COST_COUT, force_general=False, threads=1) -> Memo:
    """MPDP: Alg. 2 when the join graph is a tree, else Alg. 3 (n <= 30).
    A query with ``base_cost`` set treats relation v as an intermediate
    result whose plan costs base_cost[v].  ``threads`` > 1 splits the sets
    of each level over that many threads (same memo and counters)."""
    bc = getattr(q, "base_cost", None)
    if bc is not None:
        if force_general or threads != 1:
            raise ValueError("force_general and threads are not combined with base costs")
        b = np.ascontiguousarray(bc, dtype=np.float64)
        return _run(lib().oracle_mpdp_bc, q, cost_model, _p(b, ctypes.c_double))
    if threads != 1:
        return _run(lib().oracle_mpdp_threads, q, cost_model, int(bool(force_general)), int(threads))
    return _run(lib().oracle_mpdp, q, cost_model, int(bool(force_general)))


def dpccp(q, cost_model=COST_COUT) -> Memo:
    """DPccp csg-cmp pairs, bucketed by result size, then the DP (n <= 26)."""
    return _run(lib().oracle_dpccp, q, cost_model)


def count_ccp(q) -> int:
    """Unordered csg-cmp pairs of the whole join graph (DPccp enumeration)."""
    e, _, _ = _inputs(q)
    return int(lib().oracle_count_ccp(q.n, q.m, _p(e, ctypes.c_uint32)))


def card(q, S: int) -> float:
    e, c, s = _inputs(q)
    out = ctypes.c_double()
    rc = lib().oracle_card(q.n, q.m, _p(e, ctypes.c_uint32), _p(c, ctypes.c_double),
                           _p(s, ctypes.c_double), ctypes.c_uint32(S), ctypes.byref(out))
    if rc:
        raise ValueError("bad query")
    return out.value


def grow(q, source: int, restriction: int) -> int:
    e, _, _ = _inputs(q)
    return int(lib().oracle_grow(q.n, q.m, _p(e, ctypes.c_uint32), source, restriction))


def blocks(q, S: int) -> list[int]:
    e, _, _ = _inputs(q)
    out = np.zeros(32, np.uint32)
    k = lib().oracle_blocks(q.n, q.m, _p(e, ctypes.c_uint32), S, _p(out, ctypes.c_uint32))
    if k < 0:
        raise ValueError("bad query")
    return sorted(int(x) for x in out[:k])


def mpdp_candidates(q, S: int) -> int:
    """Alg. 3 candidate pairs for one set: sum over blocks of 2^b - 2."""
    e, _, _ = _inputs(q)
    return int(lib().oracle_mpdp_candidates(q.n, q.m, _p(e, ctypes.c_uint32), S))


def plan_from_memo(memo: Memo) -> list[dict]:
    """Plan tree from the memo (Section 5: the best plan is fetched
    recursively through left/right).  Nodes 0..n-1 are the base relations in
    index order; join nodes follow in post-order; the root comes last."""
    n = memo.n
    nodes = [dict(relset=1 << v, left=-1, right=-1, op=OP_SCAN,
                  cost=float(memo.cost[1 << v]), card=float(memo.card[1 << v])) for v in range(n)]

    def rec(S: int) -> int:
        if S & (S - 1) == 0:
            return S.bit_length() - 1
        L = int(memo.left[S])
        if L == 0 or (L & ~S) or L == S:
            raise ValueError(f"no plan for set {S:#x}")
        a = rec(L)
        b = rec(S & ~L)
        nodes.append(dict(relset=S, left=a, right=b, op=int(memo.op[S]),
                          cost=float(memo.cost[S]), card=float(memo.card[S])))
        return len(nodes) - 1

    rec(memo.full)
    return nodes


def induced(q, S: int):
    """The sub-query on the relations of S, relabelled in increasing order.
    The relabelling keeps the order of relations, so card(), the cost
    formulas and the left-bitmap tie-break give the same values for subsets
    of S: the sub-query's root entry equals the full query's memo entry of S."""
    from paper_2202_13511_amd.workloads import Query
    rel = [v for v in range(q.n) if S >> v & 1]
    pos = {v: i for i, v in enumerate(rel)}
    keep = [i for i, (u, v) in enumerate(q.edges.tolist()) if u in pos and v in pos]
    e = np.array([[pos[int(q.edges[i, 0])], pos[int(q.edges[i, 1])]] for i in keep], np.uint32).reshape(-1, 2)
    return Query(len(rel), e, q.card[rel].copy(), q.sel[keep].copy(), f"{q.name}[{S:#x}]"), rel


def expand(rel, local: int) -> int:
    """Map a relation set of an induced sub-query back to the full query."""
    out = 0
    for i, v in enumerate(rel):
        if local >> i & 1:
            out |= 1 << v
    return out


def recost_plan(q, plan, cost_model):
    """Cost of a plan (list of mpdp_plan_node-like dicts: leaves first, root
    last) recomputed bottom-up from its own nodes with card() and the written
    cost definitions; also checks every join node joins a csg-cmp pair."""
    cost, crd = {}, {}
    for i, nd in enumerate(plan):
        if nd["left"] < 0:
            v = nd["relset"].bit_length() - 1
            cost[i] = 0.01 * float(q.card[v]) if cost_model == COST_PGLIKE else 0.0
            crd[i] = float(q.card[v])
            continue
        a, b = nd["left"], nd["right"]
        L, R = plan[a]["relset"], plan[b]["relset"]
        if L & R or (L | R) != nd["relset"]:
            raise ValueError("children do not partition the node")
        for X in (L, R):
            if grow(q, X & -X, X) != X:
                raise ValueError("child not connected")
        if grow(q, L, L | R) != L | R:
            raise ValueError("children not adjacent")
        cS = card(q, nd["relset"])
        crd[i] = cS
        if cost_model == COST_COUT:
            cost[i] = (cost[a] + cost[b]) + cS
        elif nd["op"] == OP_HASH:
            cost[i] = (((cost[a] + cost[b]) + 0.0125 * crd[b]) + 0.0025 * crd[a]) + 0.01 * cS
        else:
            cost[i] = ((cost[a] + cost[b]) + (0.0025 * crd[a]) * crd[b]) + 0.01 * cS
    return cost[len(plan) - 1]
