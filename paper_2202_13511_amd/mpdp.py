"""Python binding of the C-ABI in include/mpdp.h (argument marshalling only).

Every step of the optimizer runs in the HIP library ``libmpdp.so`` built from
``csrc/``; this module converts arrays, calls the entry points with the same
names, and turns the results into Python objects.  PyTorch is used only to
own the device workspace and to name the stream.  If the library is missing
the import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpdp.so")

MPDP_OK, MPDP_EINVAL, MPDP_ENOTCONNECTED, MPDP_ETOOLARGE, MPDP_ENOMEM, MPDP_EDEVICE, MPDP_ETIMEOUT = range(7)
MPDP_COST_COUT, MPDP_COST_PGLIKE = 0, 1
MPDP_OP_SCAN, MPDP_OP_HASH, MPDP_OP_NESTLOOP, MPDP_OP_JOIN = 0, 1, 2, 3
MPDP_FLAG_TIMING = 1
MPDP_FLAG_ABLATE_DPSUB, MPDP_FLAG_ABLATE_NO_COMPACTION, MPDP_FLAG_ABLATE_UNFUSED_PRUNE = 2, 4, 8
_FLAG_FORCE_GENERAL = 0x100   # test aid: block-based kernel on tree joins too
_FLAG_BATCH_ALL_TEAMS = 0x200  # test aid: every batched query that may take a team of workgroups takes one

EXPORTED = ["mpdp_status_str", "mpdp_workspace_bytes", "mpdp_memo_layout", "mpdp_optimize",
            "mpdp_optimize_ws", "mpdp_noalloc_scratch_bytes", "mpdp_optimize_noalloc", "mpdp_optimize_units", "mpdp_optimize_cpu", "mpdp_batch_workspace_bytes", "mpdp_optimize_batch",
            "mpdp_optimize_batch_sched", "mpdp_batch_autotune", "mpdp_batch_graph_create", "mpdp_batch_graph_run",
            "mpdp_batch_graph_destroy",
            "mpdp_optimize_large", "mpdp_optimize_large_budget", "mpdp_large_examples", "mpdp_scorer_param_bytes", "mpdp_scorer_work_bytes", "mpdp_scorer_layout",
            "mpdp_scorer_load", "mpdp_scorer_forward", "mpdp_scorer_grad", "mpdp_scorer_train_step"]
SCORER_IN, SCORER_HIDDEN = 32, 256
MPDP_LARGE_GOO, MPDP_LARGE_IDP2, MPDP_LARGE_UNIONDP, MPDP_LARGE_UNIONDP_LEARNED = 0, 1, 2, 3


class mpdp_edge(ctypes.Structure):
    _fields_ = [("u", ctypes.c_uint32), ("v", ctypes.c_uint32)]


class mpdp_plan_node(ctypes.Structure):
    _fields_ = [("left", ctypes.c_int32), ("right", ctypes.c_int32), ("relset", ctypes.c_uint32),
                ("op", ctypes.c_uint32), ("cost", ctypes.c_double), ("card", ctypes.c_double)]


class mpdp_stats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_uint64), ("connected_sets", ctypes.c_uint64),
                ("evaluated_pairs", ctypes.c_uint64), ("ccp_pairs", ctypes.c_uint64),
                ("ms_total", ctypes.c_double), ("ms_filter", ctypes.c_double),
                ("ms_eval", ctypes.c_double), ("levels", ctypes.c_uint32),
                ("eval_launches", ctypes.c_uint32)]


class mpdp_batch_query(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint32), ("card_offset", ctypes.c_uint32),
                ("edge_offset", ctypes.c_uint32)]


class mpdp_batch_schedule(ctypes.Structure):
    _fields_ = [("tree_chunk", ctypes.c_uint32), ("heavy_chunks", ctypes.c_uint32)]


class mpdp_batch_tune_stats(ctypes.Structure):
    _fields_ = [("classes", ctypes.c_uint32), ("launches", ctypes.c_uint32), ("ms_total", ctypes.c_double),
                ("est_default_ms", ctypes.c_double), ("est_tuned_ms", ctypes.c_double)]


class mpdp_batch_stats(ctypes.Structure):
    _fields_ = [("connected_sets", ctypes.c_uint64), ("evaluated_pairs", ctypes.c_uint64),
                ("ccp_pairs", ctypes.c_uint64), ("ms_total", ctypes.c_double), ("ms_kernel", ctypes.c_double),
                ("workgroups", ctypes.c_uint32), ("max_n", ctypes.c_uint32)]


class mpdp_large_node(ctypes.Structure):
    _fields_ = [("left", ctypes.c_int32), ("right", ctypes.c_int32), ("rel", ctypes.c_uint32),
                ("nrels", ctypes.c_uint32), ("op", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("cost", ctypes.c_double), ("card", ctypes.c_double)]


class mpdp_large_stats(ctypes.Structure):
    _fields_ = [("exact_calls", ctypes.c_uint64), ("exact_units", ctypes.c_uint64),
                ("max_units", ctypes.c_uint32), ("rounds", ctypes.c_uint32), ("launches", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("ms_total", ctypes.c_double), ("ms_exact", ctypes.c_double)]


class MpdpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mpdp status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libmpdp.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2202_13511_amd.build.build()")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one this library links.  Loading torch first makes both use that one
    # runtime; the other order leaves torch unable to initialise the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    u32, sz, vp = ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p
    f64p = ctypes.POINTER(ctypes.c_double)
    L.mpdp_status_str.argtypes = [ctypes.c_int]
    L.mpdp_status_str.restype = ctypes.c_char_p
    L.mpdp_workspace_bytes.argtypes = [u32, ctypes.c_int]
    L.mpdp_workspace_bytes.restype = sz
    L.mpdp_memo_layout.argtypes = [u32] + [ctypes.POINTER(sz)] * 4
    L.mpdp_memo_layout.restype = ctypes.c_int
    common = [u32, u32, ctypes.POINTER(mpdp_edge), f64p, f64p, ctypes.c_int]
    outs = [ctypes.POINTER(mpdp_plan_node), f64p, ctypes.POINTER(mpdp_stats)]
    L.mpdp_optimize.argtypes = common + outs
    L.mpdp_optimize.restype = ctypes.c_int
    L.mpdp_optimize_ws.argtypes = common + [vp, sz, vp, u32] + outs
    L.mpdp_optimize_ws.restype = ctypes.c_int
    L.mpdp_noalloc_scratch_bytes.argtypes = []
    L.mpdp_noalloc_scratch_bytes.restype = sz
    L.mpdp_optimize_noalloc.argtypes = common + [vp, u32] + outs
    L.mpdp_optimize_noalloc.restype = ctypes.c_int
    L.mpdp_optimize_cpu.argtypes = common + [u32] + outs
    L.mpdp_optimize_cpu.restype = ctypes.c_int
    L.mpdp_optimize_units.argtypes = common[:5] + [f64p, ctypes.c_int, vp, sz, vp, u32] + outs
    L.mpdp_optimize_units.restype = ctypes.c_int
    L.mpdp_optimize_large.argtypes = common + [ctypes.c_int, u32, vp, vp, ctypes.POINTER(mpdp_large_node), f64p,
                                               ctypes.POINTER(mpdp_large_stats)]
    L.mpdp_large_examples.argtypes = common + [u32, vp, ctypes.POINTER(ctypes.c_uint32), u32, vp, vp,
                                               ctypes.POINTER(ctypes.c_float), u32, ctypes.POINTER(ctypes.c_uint32)]
    L.mpdp_large_examples.restype = ctypes.c_int
    L.mpdp_optimize_large.restype = ctypes.c_int
    L.mpdp_optimize_large_budget.argtypes = common + [ctypes.c_int, u32, vp, ctypes.c_double, vp,
                                                      ctypes.POINTER(mpdp_large_node), f64p,
                                                      ctypes.POINTER(mpdp_large_stats)]
    L.mpdp_optimize_large_budget.restype = ctypes.c_int
    L.mpdp_scorer_param_bytes.argtypes = []
    L.mpdp_scorer_param_bytes.restype = sz
    L.mpdp_scorer_work_bytes.argtypes = [u32]
    L.mpdp_scorer_work_bytes.restype = sz
    L.mpdp_scorer_layout.argtypes = [ctypes.POINTER(sz)] * 3
    L.mpdp_scorer_layout.restype = ctypes.c_int
    f32p = ctypes.POINTER(ctypes.c_float)
    L.mpdp_scorer_load.argtypes = [vp] + [f32p] * 6 + [vp]
    L.mpdp_scorer_load.restype = ctypes.c_int
    L.mpdp_scorer_forward.argtypes = [vp, vp, u32, vp, vp, sz, vp]
    L.mpdp_scorer_forward.restype = ctypes.c_int
    L.mpdp_scorer_grad.argtypes = [vp, vp, vp, u32, vp, sz, vp, f32p]
    L.mpdp_scorer_grad.restype = ctypes.c_int
    L.mpdp_scorer_train_step.argtypes = [vp, vp, vp, u32, ctypes.c_float, u32, vp, sz, vp, f32p]
    L.mpdp_scorer_train_step.restype = ctypes.c_int
    bq = ctypes.POINTER(mpdp_batch_query)
    L.mpdp_batch_workspace_bytes.argtypes = [u32, bq]
    L.mpdp_batch_workspace_bytes.restype = sz
    L.mpdp_optimize_batch.argtypes = [u32, bq, ctypes.POINTER(mpdp_edge), f64p, f64p, ctypes.c_int, vp, sz, vp,
                                      u32, ctypes.POINTER(mpdp_plan_node), f64p, f64p, f64p,
                                      ctypes.POINTER(mpdp_batch_stats)]
    L.mpdp_optimize_batch.restype = ctypes.c_int
    sch = ctypes.POINTER(mpdp_batch_schedule)
    L.mpdp_optimize_batch_sched.argtypes = [u32, bq, ctypes.POINTER(mpdp_edge), f64p, f64p, ctypes.c_int, vp, sz, vp,
                                            u32, sch, ctypes.POINTER(mpdp_plan_node), f64p, f64p, f64p,
                                            ctypes.POINTER(mpdp_batch_stats)]
    L.mpdp_optimize_batch_sched.restype = ctypes.c_int
    L.mpdp_batch_autotune.argtypes = [u32, bq, ctypes.POINTER(mpdp_edge), f64p, f64p, ctypes.c_int, vp, sz, vp, u32,
                                      sch, ctypes.POINTER(mpdp_batch_tune_stats)]
    L.mpdp_batch_autotune.restype = ctypes.c_int
    L.mpdp_batch_graph_create.argtypes = [u32, bq, ctypes.c_int, vp, sz, ctypes.POINTER(vp)]
    L.mpdp_batch_graph_create.restype = ctypes.c_int
    L.mpdp_batch_graph_run.argtypes = [vp, bq, ctypes.POINTER(mpdp_edge), f64p, f64p, sch, vp,
                                       ctypes.POINTER(mpdp_plan_node), f64p, f64p, ctypes.POINTER(mpdp_batch_stats)]
    L.mpdp_batch_graph_run.restype = ctypes.c_int
    L.mpdp_batch_graph_destroy.argtypes = [vp]
    L.mpdp_batch_graph_destroy.restype = None
    _lib = L
    return L


@dataclass
class Result:
    cost: float
    plan: list            # list of dicts, layout of mpdp_plan_node
    stats: dict

    def plan_array(self) -> np.ndarray:
        return np.array([(p["left"], p["right"], p["relset"], p["op"], p["cost"], p["card"])
                         for p in self.plan],
                        dtype=[("left", "i4"), ("right", "i4"), ("relset", "u4"), ("op", "u4"),
                               ("cost", "f8"), ("card", "f8")])


def mpdp_status_str(status: int) -> str:
    return load().mpdp_status_str(int(status)).decode()


def mpdp_workspace_bytes(n: int, cost_model: int = MPDP_COST_COUT) -> int:
    return int(load().mpdp_workspace_bytes(int(n), int(cost_model)))


def mpdp_memo_layout(n: int) -> dict:
    o = [ctypes.c_size_t() for _ in range(4)]
    st = load().mpdp_memo_layout(int(n), *[ctypes.byref(x) for x in o])
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))
    return dict(cost=o[0].value, card=o[1].value, left=o[2].value, op=o[3].value)


def _marshal(n, edges, card, sel):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.uint32).reshape(-1, 2))
    c = np.ascontiguousarray(np.asarray(card, dtype=np.float64))
    s = np.ascontiguousarray(np.asarray(sel, dtype=np.float64))
    m = e.shape[0]
    ep = e.ctypes.data_as(ctypes.POINTER(mpdp_edge)) if m else None
    cp = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if c.size else None
    sp = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if s.size else None
    return (e, c, s), m, ep, cp, sp


def _result(n, plan, cost, stats) -> Result:
    nodes = [dict(left=p.left, right=p.right, relset=p.relset, op=p.op, cost=p.cost, card=p.card)
             for p in plan[: 2 * n - 1]]
    st = {f: getattr(stats, f) for f, _ in mpdp_stats._fields_}
    return Result(cost.value, nodes, st)


def _args(query):
    return query.n, query.edges, query.card, query.sel


def mpdp_optimize(query, cost_model: int = MPDP_COST_COUT) -> Result:
    """Self-contained call: the library allocates its own workspace."""
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    plan = (mpdp_plan_node * max(2 * n - 1, 1))()
    cost = ctypes.c_double()
    stats = mpdp_stats()
    st = load().mpdp_optimize(int(n), m, ep, cp, sp, int(cost_model), plan, ctypes.byref(cost),
                              ctypes.byref(stats))
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))
    return _result(n, plan, cost, stats)


def mpdp_optimize_cpu(query, cost_model: int = MPDP_COST_COUT, threads: int = 0) -> Result:
    """The exact DP on the host's cores (threads = 0: all hardware threads)."""
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    plan = (mpdp_plan_node * max(2 * n - 1, 1))()
    cost = ctypes.c_double()
    stats = mpdp_stats()
    st = load().mpdp_optimize_cpu(int(n), m, ep, cp, sp, int(cost_model), int(threads), plan, ctypes.byref(cost),
                                  ctypes.byref(stats))
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))
    return _result(n, plan, cost, stats)


def workspace(n: int, cost_model: int = MPDP_COST_COUT, device="cuda"):
    """A torch-owned device workspace for mpdp_optimize_ws."""
    import torch
    nbytes = mpdp_workspace_bytes(n, cost_model)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def mpdp_optimize_ws(query, cost_model: int, ws, stream=None, flags: int = 0) -> Result:
    """Run on caller-owned device memory (a torch uint8 tensor) and stream."""
    import torch
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    if stream is None:
        stream = torch.cuda.current_stream(ws.device)
    plan = (mpdp_plan_node * max(2 * n - 1, 1))()
    cost = ctypes.c_double()
    stats = mpdp_stats()
    st = load().mpdp_optimize_ws(int(n), m, ep, cp, sp, int(cost_model), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel() * ws.element_size(), ctypes.c_void_p(stream.cuda_stream),
                                 int(flags), plan, ctypes.byref(cost), ctypes.byref(stats))
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))
    return _result(n, plan, cost, stats)


MPDP_NOALLOC_MAX_REL = 20


def mpdp_noalloc_scratch_bytes() -> int:
    return int(load().mpdp_noalloc_scratch_bytes())


def mpdp_optimize_noalloc(query, cost_model: int, stream=None, flags: int = 0) -> Result:
    """mpdp_optimize_ws without a workspace: the library's fixed device array
    (n <= MPDP_NOALLOC_MAX_REL); nothing is allocated by the call."""
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    sp_handle = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    plan = (mpdp_plan_node * max(2 * n - 1, 1))()
    cost = ctypes.c_double()
    stats = mpdp_stats()
    st = load().mpdp_optimize_noalloc(int(n), m, ep, cp, sp, int(cost_model), sp_handle, int(flags), plan,
                                      ctypes.byref(cost), ctypes.byref(stats))
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))
    return _result(n, plan, cost, stats)


def mpdp_optimize_units(query, cost_model: int, ws, stream=None, flags: int = 0) -> Result:
    """mpdp_optimize_ws for a query whose relations are planned intermediate
    results: ``query.base_cost[v]`` is the cost of relation v's plan."""
    import torch
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    bc = np.ascontiguousarray(np.asarray(query.base_cost, dtype=np.float64))
    if stream is None:
        stream = torch.cuda.current_stream(ws.device)
    plan = (mpdp_plan_node * max(2 * n - 1, 1))()
    cost = ctypes.c_double()
    stats = mpdp_stats()
    st = load().mpdp_optimize_units(int(n), m, ep, cp, sp, bc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    int(cost_model), ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                    ctypes.c_void_p(stream.cuda_stream), int(flags), plan, ctypes.byref(cost),
                                    ctypes.byref(stats))
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))
    return _result(n, plan, cost, stats)


@dataclass
class LargeResult:
    cost: float
    plan: list            # list of dicts, layout of mpdp_large_node
    stats: dict


def mpdp_optimize_large(query, cost_model: int, method: int, k: int, scorer=None, stream=None,
                        budget_ms: float | None = None) -> LargeResult:
    """Large-query heuristics (GOO, IDP2, UnionDP, learned UnionDP) with the
    exact DP on the GPU as the inner step; the library owns its device
    workspace.  scorer: a device parameter block (scorer_params()).
    budget_ms: a wall-clock budget (mpdp_optimize_large_budget); a run that
    exhausts it returns the plan found so far with stats["timed_out"] set."""
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    plan = (mpdp_large_node * max(2 * n - 1, 1))()
    cost = ctypes.c_double()
    stats = mpdp_large_stats()
    sp_handle = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    sc = None if scorer is None else ctypes.c_void_p(scorer.data_ptr())
    if budget_ms is None:
        st = load().mpdp_optimize_large(int(n), m, ep, cp, sp, int(cost_model), int(method), int(k), sc,
                                        sp_handle, plan, ctypes.byref(cost), ctypes.byref(stats))
    else:
        st = load().mpdp_optimize_large_budget(int(n), m, ep, cp, sp, int(cost_model), int(method), int(k), sc,
                                               float(budget_ms), sp_handle, plan, ctypes.byref(cost),
                                               ctypes.byref(stats))
    if st not in (MPDP_OK, MPDP_ETIMEOUT):
        raise MpdpError(st, mpdp_status_str(st))
    nodes = [dict(left=p.left, right=p.right, rel=p.rel, nrels=p.nrels, op=p.op, cost=p.cost, card=p.card)
             for p in plan[: 2 * n - 1]]
    info = {f: getattr(stats, f) for f, _ in mpdp_large_stats._fields_}
    info["timed_out"] = st == MPDP_ETIMEOUT
    return LargeResult(cost.value, nodes, info)


def mpdp_large_examples(query, cost_model: int, k: int, plan_sets, scorer=None, stream=None):
    """(features (rows, 32) uint16 bfloat16 bits, labels (rows,) float32) of
    UnionDP's candidate unions on a query of n <= 32 relations whose optimal
    plan has the relation sets `plan_sets`."""
    n, edges, card, sel = _args(query)
    keep, m, ep, cp, sp = _marshal(n, edges, card, sel)
    sets = np.ascontiguousarray(np.asarray(sorted(plan_sets), np.uint32))
    sc = None if scorer is None else ctypes.c_void_p(scorer.data_ptr())
    sp_handle = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    cap = 4096
    while True:
        X = np.zeros((cap, SCORER_IN), np.uint16)
        y = np.zeros(cap, np.float32)
        cnt = ctypes.c_uint32()
        st = load().mpdp_large_examples(int(n), m, ep, cp, sp, int(cost_model), int(k), sc,
                                        sets.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(sets), sp_handle,
                                        ctypes.c_void_p(X.ctypes.data), y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        cap, ctypes.byref(cnt))
        if st == MPDP_ENOMEM and cnt.value > cap:
            cap = int(cnt.value)
            continue
        _check(st)
        return X[: cnt.value], y[: cnt.value]


def memo_index(n: int) -> np.ndarray:
    """Memo index of every relation-set bitmap S < 2^n under the level-compact
    layout documented at mpdp_memo_layout: off(|S|) + colex(S)."""
    from math import comb
    S = np.arange(1 << n, dtype=np.uint64)
    pop = np.zeros(1 << n, dtype=np.int64)
    rank = np.zeros(1 << n, dtype=np.uint64)
    for v in range(n):
        has = ((S >> np.uint64(v)) & np.uint64(1)).astype(bool)
        table = np.array([comb(v, p + 1) for p in range(n + 1)], dtype=np.uint64)
        rank[has] += table[pop[has]]
        pop += has
    off = np.zeros(n + 2, dtype=np.uint64)
    for k in range(1, n + 2):
        off[k] = off[k - 1] + np.uint64(comb(n, k - 1))
    return off[pop] + rank


def memo_arrays(ws, n: int) -> dict:
    """Host copies of the memo arrays left in a workspace by mpdp_optimize_ws,
    re-indexed by relation-set bitmap (entry S at position S)."""
    lay = mpdp_memo_layout(n)
    N = 1 << n
    idx = memo_index(n)
    out = {}
    for name, dt, width in (("cost", np.float64, 8), ("card", np.float64, 8), ("left", np.uint32, 4),
                            ("op", np.uint8, 1)):
        seg = ws[lay[name]: lay[name] + N * width].cpu().numpy().view(dt)
        out[name] = seg[idx]
    return out


@dataclass
class BatchResult:
    costs: list           # root cost per query
    plans: list           # per query: list of plan-node dicts (layout of mpdp_plan_node)
    latency_us: np.ndarray
    stats: dict
    start_us: np.ndarray = None


def _batch_marshal(queries):
    qs = (mpdp_batch_query * len(queries))()
    cards, edges, sels = [], [], []
    co = eo = 0
    for i, q in enumerate(queries):
        qs[i] = mpdp_batch_query(q.n, q.m, co, eo)
        cards.append(np.asarray(q.card, np.float64))
        edges.append(np.asarray(q.edges, np.uint32).reshape(-1, 2))
        sels.append(np.asarray(q.sel, np.float64))
        co += q.n
        eo += q.m
    c = np.ascontiguousarray(np.concatenate(cards))
    e = np.ascontiguousarray(np.concatenate(edges)) if eo else np.zeros((1, 2), np.uint32)
    s = np.ascontiguousarray(np.concatenate(sels)) if eo else np.zeros(1, np.float64)
    return qs, c, e, s


def mpdp_batch_workspace_bytes(queries) -> int:
    qs, _, _, _ = _batch_marshal(queries)
    return int(load().mpdp_batch_workspace_bytes(len(queries), qs))


def batch_workspace(queries, device="cuda"):
    import torch
    return torch.empty(max(mpdp_batch_workspace_bytes(queries), 256), dtype=torch.uint8, device=device)


def _split_plans(queries, plans):
    out, at = [], 0
    for q in queries:
        k = 2 * q.n - 1
        out.append([dict(left=p.left, right=p.right, relset=p.relset, op=p.op, cost=p.cost, card=p.card)
                    for p in plans[at: at + k]])
        at += k
    return out


def _schedules(queries, schedules):
    """None, or one (tree_chunk, heavy_chunks) pair per query."""
    if schedules is None:
        return None
    arr = (mpdp_batch_schedule * len(queries))()
    for i, (tc, hc) in enumerate(schedules):
        arr[i] = mpdp_batch_schedule(int(tc), int(hc))
    return arr


def mpdp_optimize_batch(queries, cost_model: int, ws, stream=None, flags: int = 0, schedules=None) -> BatchResult:
    """All queries (n <= 20 each) in one persistent launch; `schedules`, if
    given, holds one (tree_chunk, heavy_chunks) pair per query."""
    import torch
    qs, c, e, s = _batch_marshal(queries)
    if stream is None:
        stream = torch.cuda.current_stream(ws.device)
    total = sum(2 * q.n - 1 for q in queries)
    plans = (mpdp_plan_node * total)()
    costs = np.zeros(len(queries), np.float64)
    lat = np.zeros(len(queries), np.float64)
    start = np.zeros(len(queries), np.float64)
    st = mpdp_batch_stats()
    f64p = ctypes.POINTER(ctypes.c_double)
    args = [len(queries), qs, e.ctypes.data_as(ctypes.POINTER(mpdp_edge)), c.ctypes.data_as(f64p),
            s.ctypes.data_as(f64p), int(cost_model), ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
            ctypes.c_void_p(stream.cuda_stream), int(flags)]
    tail = [plans, costs.ctypes.data_as(f64p), lat.ctypes.data_as(f64p), start.ctypes.data_as(f64p), ctypes.byref(st)]
    sch = _schedules(queries, schedules)
    if sch is None:
        rc = load().mpdp_optimize_batch(*args, *tail)
    else:
        rc = load().mpdp_optimize_batch_sched(*args, sch, *tail)
    if rc != MPDP_OK:
        raise MpdpError(rc, mpdp_status_str(rc))
    return BatchResult(costs.tolist(), _split_plans(queries, plans), lat,
                       {f: getattr(st, f) for f, _ in mpdp_batch_stats._fields_}, start)


def mpdp_batch_autotune(queries, cost_model: int, ws, reps: int = 2, stream=None):
    """Per-query schedules chosen by the library's autotuner: returns
    ([(tree_chunk, heavy_chunks)] per query, stats dict)."""
    import torch
    qs, c, e, s = _batch_marshal(queries)
    if stream is None:
        stream = torch.cuda.current_stream(ws.device)
    out = (mpdp_batch_schedule * len(queries))()
    st = mpdp_batch_tune_stats()
    f64p = ctypes.POINTER(ctypes.c_double)
    rc = load().mpdp_batch_autotune(len(queries), qs, e.ctypes.data_as(ctypes.POINTER(mpdp_edge)),
                                    c.ctypes.data_as(f64p), s.ctypes.data_as(f64p), int(cost_model),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                    ctypes.c_void_p(stream.cuda_stream), int(reps), out, ctypes.byref(st))
    if rc != MPDP_OK:
        raise MpdpError(rc, mpdp_status_str(rc))
    return ([(o.tree_chunk, o.heavy_chunks) for o in out],
            {f: getattr(st, f) for f, _ in mpdp_batch_tune_stats._fields_})


class BatchGraph:
    """A batch shape captured once in a HIP graph (mpdp_batch_graph_*) and
    replayed with the data of any batch of that shape."""

    def __init__(self, queries, cost_model: int, ws):
        qs, _, _, _ = _batch_marshal(queries)
        self.shape = [(q.n, q.m) for q in queries]
        self.cost_model = int(cost_model)
        self.ws = ws  # the workspace must outlive the graph
        h = ctypes.c_void_p()
        rc = load().mpdp_batch_graph_create(len(queries), qs, self.cost_model, ctypes.c_void_p(ws.data_ptr()),
                                            ws.numel() * ws.element_size(), ctypes.byref(h))
        if rc != MPDP_OK:
            raise MpdpError(rc, mpdp_status_str(rc))
        self.handle = h

    def run(self, queries, schedules=None, stream=None) -> BatchResult:
        import torch
        if self.handle is None:
            raise MpdpError(MPDP_EINVAL, "graph destroyed")
        qs, c, e, s = _batch_marshal(queries)
        if stream is None:
            stream = torch.cuda.current_stream(self.ws.device)
        total = sum(2 * q.n - 1 for q in queries)
        plans = (mpdp_plan_node * total)()
        costs = np.zeros(len(queries), np.float64)
        lat = np.zeros(len(queries), np.float64)
        st = mpdp_batch_stats()
        f64p = ctypes.POINTER(ctypes.c_double)
        rc = load().mpdp_batch_graph_run(self.handle, qs, e.ctypes.data_as(ctypes.POINTER(mpdp_edge)),
                                         c.ctypes.data_as(f64p), s.ctypes.data_as(f64p),
                                         _schedules(queries, schedules), ctypes.c_void_p(stream.cuda_stream), plans,
                                         costs.ctypes.data_as(f64p), lat.ctypes.data_as(f64p), ctypes.byref(st))
        if rc != MPDP_OK:
            raise MpdpError(rc, mpdp_status_str(rc))
        return BatchResult(costs.tolist(), _split_plans(queries, plans), lat,
                           {f: getattr(st, f) for f, _ in mpdp_batch_stats._fields_})

    def close(self):
        if self.handle is not None:
            load().mpdp_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned scorer (mpdp_scorer.h)

_SCORER_SHAPES = (("w1", (SCORER_IN, SCORER_HIDDEN)), ("b1", (SCORER_HIDDEN,)), ("w2", (SCORER_HIDDEN, SCORER_HIDDEN)),
                  ("b2", (SCORER_HIDDEN,)), ("w3", (SCORER_HIDDEN,)), ("b3", (1,)))


def _check(st):
    if st != MPDP_OK:
        raise MpdpError(st, mpdp_status_str(st))


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(dev, stream):
    import torch
    return ctypes.c_void_p((stream or torch.cuda.current_stream(dev)).cuda_stream)


def scorer_params(device="cuda"):
    """A torch-owned device parameter block."""
    import torch
    return torch.zeros(int(load().mpdp_scorer_param_bytes()), dtype=torch.uint8, device=device)


def scorer_work(batch: int, device="cuda"):
    import torch
    return torch.zeros(max(int(load().mpdp_scorer_work_bytes(int(batch))), 256), dtype=torch.uint8, device=device)


def scorer_load(block, weights: dict, stream=None):
    arrs = [np.ascontiguousarray(np.asarray(weights[k], np.float32).reshape(shape)) for k, shape in _SCORER_SHAPES]
    f32p = ctypes.POINTER(ctypes.c_float)
    _check(load().mpdp_scorer_load(_dev(block), *[a.ctypes.data_as(f32p) for a in arrs], _stream(block.device, stream)))


def _scorer_region(block, which: str) -> dict:
    """FP32 master values ('master') or gradients ('grad') as numpy arrays."""
    import torch
    o = [ctypes.c_size_t() for _ in range(3)]
    _check(load().mpdp_scorer_layout(*[ctypes.byref(x) for x in o]))
    off = o[0].value if which == "master" else o[2].value
    total = sum(int(np.prod(sh)) for _, sh in _SCORER_SHAPES)
    torch.cuda.synchronize(block.device)
    flat = block[off: off + 4 * total].view(torch.float32).cpu().numpy().astype(np.float32)
    out, at = {}, 0
    for k, sh in _SCORER_SHAPES:
        n = int(np.prod(sh))
        out[k] = flat[at: at + n].reshape(sh)
        at += n
    return out


def scorer_weights(block) -> dict:
    return _scorer_region(block, "master")


def scorer_grads(block) -> dict:
    return _scorer_region(block, "grad")


def scorer_forward(block, x_bits, work=None, stream=None) -> np.ndarray:
    """Logits of a batch; x_bits: (B, 32) uint16 bfloat16 bit patterns (numpy or torch int16 on the device)."""
    import torch
    x = _to_device_bits(x_bits, block.device)
    B = x.shape[0]
    work = work if work is not None else scorer_work(B, block.device)
    out = torch.empty(B, dtype=torch.float32, device=block.device)
    _check(load().mpdp_scorer_forward(_dev(block), _dev(x), B, _dev(out), _dev(work), work.numel(),
                                      _stream(block.device, stream)))
    return out.cpu().numpy()


def _to_device_bits(x_bits, device):
    import torch
    if isinstance(x_bits, torch.Tensor):
        return x_bits.contiguous()
    a = np.ascontiguousarray(np.asarray(x_bits, np.uint16)).view(np.int16)
    return torch.from_numpy(a).to(device)


def _to_device_f32(y, device):
    import torch
    if isinstance(y, torch.Tensor):
        return y.contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(y, np.float32))).to(device)


def scorer_grad(block, x_bits, y, work=None, stream=None) -> float:
    x = _to_device_bits(x_bits, block.device)
    yy = _to_device_f32(y, block.device)
    B = x.shape[0]
    work = work if work is not None else scorer_work(B, block.device)
    loss = ctypes.c_float()
    _check(load().mpdp_scorer_grad(_dev(block), _dev(x), _dev(yy), B, _dev(work), work.numel(),
                                   _stream(block.device, stream), ctypes.byref(loss)))
    return float(loss.value)


def scorer_train_step(block, x_bits, y, lr: float, step: int, work=None, stream=None, want_loss=True) -> float:
    x = _to_device_bits(x_bits, block.device)
    yy = _to_device_f32(y, block.device)
    B = x.shape[0]
    work = work if work is not None else scorer_work(B, block.device)
    loss = ctypes.c_float()
    _check(load().mpdp_scorer_train_step(_dev(block), _dev(x), _dev(yy), B, float(lr), int(step), _dev(work),
                                         work.numel(), _stream(block.device, stream),
                                         ctypes.byref(loss) if want_loss else None))
    return float(loss.value)
